// sw_text.hpp -- the steps around the sort on gfx950: raw text to the word
// list (first pre-processing phase, section 3) and the sorted word list back
// to text (section 4: the merged result is printed).
//
// Tokenizing.  A word is a run of bytes between ASCII whitespace (tab, line
// feed, vertical tab, form feed, carriage return, space); inside a run only
// ASCII letters are kept, every other byte is a special character and is
// dropped without ending the run; a run without letters is no word.  A letter
// starts a word when the last byte before it that is not special is
// whitespace, or when there is none.  So the only state that crosses a chunk
// boundary is "was the last non-special byte a letter, whitespace, or was
// there none", and three passes suffice: per-block summaries (letters, word
// starts under either incoming state, outgoing state), one block scanning the
// summaries, and a write pass that knows every thread's incoming state and
// output positions.  A thread classifies its 64 bytes four at a time into bit
// masks (letters, whitespace), so counts are population counts and the word
// starts one 64-bit addition.
#pragma once

#include "sw_device.hpp"
#include "sw_bytes.hpp"

namespace sw {

constexpr int kTokNT = 256;
constexpr int kTokBytes = 64;                       // bytes per thread
constexpr uint32_t kTokBlock = kTokNT * kTokBytes;  // bytes per workgroup
constexpr uint32_t kTokFlagLower = 1u;

// outgoing state of a stretch of text: its last non-special byte
enum : uint32_t { TS_NONE = 0, TS_SPACE = 1, TS_LETTER = 2 };

struct TokSum {
  uint32_t letters;
  uint32_t starts_space;    // word starts if the state coming in is TS_SPACE or TS_NONE
  uint32_t starts_letter;   // ... if it is TS_LETTER
  uint32_t last;            // TS_*
};


// The thread's bytes [p, p + cnt) as 16 dwords (little-endian byte order);
// bytes past cnt read as 0, which is special and changes nothing.
__device__ inline void tok_load(const uint8_t* text, uint64_t p, uint32_t cnt, uint32_t (&w)[16]) {
  const uint8_t* src = text + p;
  if (cnt == (uint32_t)kTokBytes && (((uintptr_t)src) & 15u) == 0) {
    const uint4* q = (const uint4*)src;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint4 v = q[j];
      w[4 * j] = v.x;
      w[4 * j + 1] = v.y;
      w[4 * j + 2] = v.z;
      w[4 * j + 3] = v.w;
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) w[j] = 0;
  for (uint32_t b = 0; b < cnt; ++b) w[b >> 2] |= (uint32_t)src[b] << (8 * (b & 3));
}

__device__ inline TokSum tok_summary(const TokMasks& m) {
  TokSum s;
  s.letters = (uint32_t)__popcll(m.letter);
  s.starts_letter = (uint32_t)__popcll(tok_starts(m, false));
  s.starts_space = (uint32_t)__popcll(tok_starts(m, true));
  const uint64_t ns = m.letter | m.space;
  s.last = ns ? (((m.space >> (63 - __clzll(ns))) & 1ull) ? TS_SPACE : TS_LETTER) : TS_NONE;
  return s;
}

// Incoming state of every thread of the block from the threads before it:
// the last non-TS_NONE `last`, or TS_NONE if every earlier thread is all
// special.  s_last holds one entry per wave.
template <int NT>
__device__ inline uint32_t tok_carry_in_block(uint32_t last, uint32_t* s_last) {
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint64_t m = __ballot(last != TS_NONE);
  const uint64_t below = m & ((1ull << lane) - 1ull);
  const int src = below ? 63 - __clzll(below) : 0;
  const uint32_t from_wave = __shfl(last, src);
  const int hi = m ? 63 - __clzll(m) : 0;
  const uint32_t wave_last = m ? __shfl(last, hi) : TS_NONE;
  if (lane == 0) s_last[wave] = wave_last;
  __syncthreads();
  uint32_t carry = below ? from_wave : TS_NONE;
  if (carry == TS_NONE) {
    for (int v = (int)wave - 1; v >= 0; --v) {
      const uint32_t x = s_last[v];
      if (x != TS_NONE) {
        carry = x;
        break;
      }
    }
  }
  __syncthreads();
  return carry;
}

__global__ void k_tok_begin(Header* h) {
  if (threadIdx.x == 0) {
    h->status = 0;
    h->abort = 0;
    h->n_words = 0;
  }
}

// Pass 1: one summary per workgroup of kTokBlock bytes.
__global__ __launch_bounds__(kTokNT) void k_tok_sum(const uint8_t* text, uint64_t n, uint4* sums) {
  __shared__ uint32_t s_last[kTokNT / 64];
  __shared__ uint32_t s_red[kTokNT / 64][3];
  const uint64_t b = blockIdx.x;
  const uint64_t p = b * kTokBlock + (uint64_t)threadIdx.x * kTokBytes;
  const uint32_t cnt = p < n ? (uint32_t)min<uint64_t>(kTokBytes, n - p) : 0u;
  uint32_t w[16];
  tok_load(text, p, cnt, w);
  const TokSum s = tok_summary(tok_masks(w));
  const uint32_t carry = tok_carry_in_block<kTokNT>(s.last, s_last);
  // threads with no state before them inside the block depend on the block's
  // incoming state; the others are settled here
  uint32_t sp, sl;
  if (carry == TS_NONE) {
    sp = s.starts_space;
    sl = s.starts_letter;
  } else {
    sp = sl = carry == TS_LETTER ? s.starts_letter : s.starts_space;
  }
  uint32_t v0 = s.letters, v1 = sp, v2 = sl;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    v0 += __shfl_xor(v0, o);
    v1 += __shfl_xor(v1, o);
    v2 += __shfl_xor(v2, o);
  }
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  if (lane == 0) {
    s_red[wave][0] = v0;
    s_red[wave][1] = v1;
    s_red[wave][2] = v2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint4 r{0, 0, 0, TS_NONE};
    for (int v = 0; v < kTokNT / 64; ++v) {
      r.x += s_red[v][0];
      r.y += s_red[v][1];
      r.z += s_red[v][2];
      if (s_last[v] != TS_NONE) r.w = s_last[v];
    }
    sums[b] = r;
  }
}

// Pass 2 (one workgroup of 1024): incoming state, letter and word prefixes of
// every block; the totals, the capacity check and the closing offset.
template <int NT>
__global__ __launch_bounds__(NT) void k_tok_scan(Header* h, const uint4* sums, uint4* pre, uint32_t nblk,
                                                 uint32_t max_words, uint32_t* out_offsets, uint32_t* out_n_words) {
  __shared__ uint32_t s_last[NT / 64];
  __shared__ uint32_t s_tmp[NT / 64];
  __shared__ uint32_t s_carry;
  uint32_t run_l = 0, run_w = 0;   // totals of earlier chunks (same in every thread)
  if (threadIdx.x == 0) s_carry = TS_NONE;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < nblk; c0 += NT) {
    const uint32_t b = c0 + threadIdx.x;
    const uint4 s = b < nblk ? sums[b] : uint4{0, 0, 0, TS_NONE};
    const uint32_t chunk_carry = s_carry;
    uint32_t carry = tok_carry_in_block<NT>(s.w, s_last);
    if (carry == TS_NONE) carry = chunk_carry;
    const uint32_t words = b < nblk ? (carry == TS_LETTER ? s.z : s.y) : 0u;
    uint32_t tl, tw;
    const uint32_t el = block_excl_scan<NT>(s.x, s_tmp, tl);
    const uint32_t ew = block_excl_scan<NT>(words, s_tmp, tw);
    if (b < nblk) pre[b] = uint4{run_l + el, run_w + ew, carry, 0u};
    // the state leaving this chunk
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int v = NT / 64 - 1; v >= 0; --v) {
        if (s_last[v] != TS_NONE) {
          s_carry = s_last[v];
          break;
        }
      }
    }
    __syncthreads();
    run_l += tl;
    run_w += tw;
  }
  if (threadIdx.x == 0) {
    h->n_words = run_w;
    if (run_w > max_words) {
      h->status |= ST_WORKSPACE;
      h->abort = 1;
    } else {
      out_offsets[run_w] = run_l;
      *out_n_words = run_w;
    }
  }
}

// Bytes [0, len) of an LDS buffer to global memory at dst (any alignment):
// the head up to a 4-byte boundary and the tail byte by byte, the middle as
// whole dwords, consecutive threads on consecutive dwords.
template <int NT>
__device__ inline void lds_bytes_to_global(const uint8_t* src, uint32_t len, uint8_t* dst) {
  const uint32_t head = min(len, (uint32_t)((4u - ((uintptr_t)dst & 3u)) & 3u));
  const uint32_t body = (len - head) >> 2;
  for (uint32_t i = threadIdx.x; i < head; i += NT) dst[i] = src[i];
  uint32_t* d32 = (uint32_t*)(dst + head);
  for (uint32_t j = threadIdx.x; j < body; j += NT) {
    const uint8_t* q = src + head + 4 * j;
    d32[j] = (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16) | ((uint32_t)q[3] << 24);
  }
  for (uint32_t i = head + 4 * body + threadIdx.x; i < len; i += NT) dst[i] = src[i];
}

// Pass 3: every thread rescans its bytes.  Its letters go to LDS at their
// places in the workgroup's stretch of chars (laid out on the output's dword
// grid, so that the stretch is stored as whole dwords), and the offsets of
// the words that start among them to the workgroup's run of offsets in LDS;
// both are then stored in order.
__global__ __launch_bounds__(kTokNT) void k_tok_write(Header* h, const uint8_t* text, uint64_t n, const uint4* pre,
                                                      uint32_t flags, uint8_t* out_chars, uint32_t* out_offsets) {
  __shared__ uint32_t s_last[kTokNT / 64];
  __shared__ uint32_t s_tmp[kTokNT / 64];
  __shared__ uint32_t s_chr32[kTokBlock / 4 + 2];
  __shared__ uint32_t s_off[kTokBlock / 2];   // a word start needs a letter and a byte before it
  if (h->abort) return;
  uint8_t* s_chr = (uint8_t*)s_chr32;
  const uint64_t b = blockIdx.x;
  const uint64_t p = b * kTokBlock + (uint64_t)threadIdx.x * kTokBytes;
  const uint32_t cnt = p < n ? (uint32_t)min<uint64_t>(kTokBytes, n - p) : 0u;
  uint32_t w[16];
  tok_load(text, p, cnt, w);
  const TokMasks tm = tok_masks(w);
  const TokSum s = tok_summary(tm);
  const uint4 bp = pre[b];
  uint32_t carry = tok_carry_in_block<kTokNT>(s.last, s_last);
  if (carry == TS_NONE) carry = bp.z;
  const uint32_t starts = carry == TS_LETTER ? s.starts_letter : s.starts_space;
  uint32_t nl, nwd;
  const uint32_t lrel = block_excl_scan<kTokNT>(s.letters, s_tmp, nl);   // inside the workgroup
  uint32_t wpos = block_excl_scan<kTokNT>(starts, s_tmp, nwd);   // inside the workgroup
  const uint32_t head = (uint32_t)((uintptr_t)(out_chars + bp.x) & 3u);   // LDS byte of the stretch's first letter
  // a letter OR 0x20 is its lower case (lower case letters have the bit)
  const uint32_t fold = (flags & kTokFlagLower) ? 0x20202020u : 0u;
  const uint64_t st = tok_starts(tm, carry != TS_LETTER);
  uint32_t lpos = lrel;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint32_t lb = (uint32_t)(tm.letter >> (4 * j)) & 0xFu;
    if (lb == 0) continue;
    const uint32_t sb = (uint32_t)(st >> (4 * j)) & 0xFu;
    const uint32_t v = w[j] | fold;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if ((lb >> t) & 1u) {
        if ((sb >> t) & 1u) s_off[wpos++] = bp.x + lpos;
        s_chr[head + lpos++] = (uint8_t)(v >> (8 * t));
      }
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nwd; k += kTokNT) out_offsets[bp.y + k] = s_off[k];
  // the stretch [head, head + nl) of LDS to out_chars + bp.x: edge bytes one
  // by one, whole dwords in between (LDS dword k is output dword k)
  uint8_t* dst = out_chars + bp.x - head;
  const uint32_t end = head + nl;
  const uint32_t d0 = (head + 3) >> 2, d1 = end >> 2;   // whole dwords [d0, d1)
  if (d0 > d1) {
    for (uint32_t i = head + threadIdx.x; i < end; i += kTokNT) dst[i] = s_chr[i];
  } else {
    for (uint32_t i = head + threadIdx.x; i < 4 * d0; i += kTokNT) dst[i] = s_chr[i];
    uint32_t* dst32 = (uint32_t*)dst;
    for (uint32_t k = d0 + threadIdx.x; k < d1; k += kTokNT) dst32[k] = s_chr32[k];
    for (uint32_t i = 4 * d1 + threadIdx.x; i < end; i += kTokNT) dst[i] = s_chr[i];
  }
}

// ---------------------------------------------------------------- sorted text
// Word k of the output (global position k over all documents) is document d's
// word perm[k] (document-local), of length L = the bucket holding its
// document-local position.  Its bytes go to
//   text_base(d) + sum_{l<L} cnt_l*(l+s) + (k' - bo[L])*(L+s)
// where s is 1 with a separator and 0 without, cnt_l and bo are document d's
// bucket counts and offsets, and text_base(d) = chars and separators of the
// documents before d.  Every word is checked (index inside its document,
// offsets inside the word list, length equal to its bucket's) and every byte
// written is checked against the output size; a failed check sets *status
// and writes nothing for that word.
__global__ void k_mat_begin(uint32_t* status) {
  if (threadIdx.x == 0) *status = 0u;
}

// Document of output position k: the last d with doc_offsets[d] <= k.
__device__ inline uint32_t mat_doc(const uint32_t* doc_offsets, uint32_t n_docs, uint32_t k) {
  uint32_t lo = 0, hi = n_docs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (doc_offsets[mid] <= k)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The bucket of a document-local position: the last L with bo[L] <= kl.
template <class BO>
__device__ inline uint32_t mat_bucket(const BO& bo, uint32_t kl) {
  uint32_t L = 0;
#pragma unroll
  for (uint32_t step = 32; step >= 1; step >>= 1)
    if (L + step <= (uint32_t)kMaxLen && bo[L + step] <= kl) L += step;
  return L;
}

// A workgroup takes NT consecutive output positions.  The bucket table of the
// document of its first position sits in LDS (words of later documents read
// theirs from memory).  When every word of the workgroup passes its checks
// and the words' places follow each other, they are assembled in LDS and
// stored as one stretch; otherwise each good word is written on its own.
template <int NT>
__global__ __launch_bounds__(NT) void k_materialize(const uint8_t* chars, const uint32_t* offsets,
                                                    const uint32_t* doc_offsets, uint32_t n_docs, uint32_t N,
                                                    const uint32_t* perm, const uint32_t* boff, int sep,
                                                    uint8_t* out, uint32_t* status) {
  __shared__ uint8_t s_txt[NT * (kMaxLen + 1)];
  __shared__ uint64_t s_base[kNB];
  __shared__ uint32_t s_bo[kNOff];
  __shared__ uint32_t s_doc[3];
  __shared__ uint32_t s_tmp[NT / 64];
  __shared__ uint64_t s_pos0;
  const uint32_t s = sep >= 0 ? 1u : 0u;
  const uint32_t o0 = offsets[0], oN = offsets[N];
  const uint64_t out_size = (uint64_t)(oN - o0) + (uint64_t)s * N;
  for (uint32_t k0 = blockIdx.x * NT; k0 < N; k0 += gridDim.x * NT) {
    if (threadIdx.x == 0) {
      const uint32_t d = doc_offsets ? mat_doc(doc_offsets, n_docs, k0) : 0u;
      s_doc[0] = d;
      s_doc[1] = doc_offsets ? doc_offsets[d] : 0u;
      s_doc[2] = doc_offsets ? doc_offsets[d + 1] : N;
    }
    __syncthreads();
    const uint32_t d0 = s_doc[0], ds0 = s_doc[1], de0 = s_doc[2];
    if (threadIdx.x < (uint32_t)kNOff) s_bo[threadIdx.x] = boff[(size_t)d0 * kNOff + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
      // text position of each bucket of document d0 (only meaningful if its
      // offsets are in range; every word is checked below anyway)
      uint64_t pos = ds0 <= N ? (uint64_t)(offsets[ds0] - o0) + (uint64_t)s * ds0 : 0u;
      for (int L = 0; L < kNB; ++L) {
        s_base[L] = pos;
        pos += (uint64_t)(s_bo[L + 1] - s_bo[L]) * (L + s);
      }
    }
    __syncthreads();
    const uint32_t k = k0 + threadIdx.x;
    bool ok = false;
    uint64_t pos = 0;
    uint32_t L = 0, a = 0;
    if (k < N) {
      uint32_t d = d0, dstart = ds0, dend = de0;
      if (doc_offsets && !(k >= ds0 && k < de0)) {
        d = mat_doc(doc_offsets, n_docs, k);
        dstart = doc_offsets[d];
        dend = doc_offsets[d + 1];
      }
      if (dstart <= k && k < dend && dend <= N) {
        const uint32_t kl = k - dstart;
        uint32_t bL;
        if (d == d0) {
          L = mat_bucket(s_bo, kl);
          bL = s_bo[L];
          pos = s_base[L];
        } else {
          const uint32_t* bo = boff + (size_t)d * kNOff;
          L = mat_bucket(bo, kl);
          bL = bo[L];
          pos = (uint64_t)(offsets[dstart] - o0) + (uint64_t)s * dstart;
          for (uint32_t l = 0; l < L; ++l) pos += (uint64_t)(bo[l + 1] - bo[l]) * (l + s);
        }
        pos += (uint64_t)(kl - bL) * (L + s);
        const uint32_t i = perm[k];
        ok = i < dend - dstart && kl >= bL && pos + L + s <= out_size;
        if (ok) {
          a = offsets[dstart + i];
          const uint32_t e = offsets[dstart + i + 1];
          ok = a >= o0 && e <= oN && e >= a && e - a == L;
        }
      }
      if (!ok) atomicOr(status, 1u);
    }
    // the word's bytes: the aligned dwords covering [a, a + L); a dword that
    // holds one of the word's bytes lies in the same page, so reading it whole
    // stays inside mapped memory
    uint32_t wv[9];
    if (ok) {
      const uint32_t* src = (const uint32_t*)((uintptr_t)(chars + a) & ~(uintptr_t)3);
      const uint32_t nd = L ? (((uintptr_t)(chars + a) & 3u) + L + 3) >> 2 : 0u;
#pragma unroll
      for (int j = 0; j < 9; ++j) wv[j] = (uint32_t)j < nd ? src[j] : 0u;
    }
    const uint32_t sh = (uint32_t)((uintptr_t)(chars + a) & 3u);
    const uint32_t size = ok ? L + s : 0u;
    uint32_t total;
    const uint32_t rel = block_excl_scan<NT>(size, s_tmp, total);
    if (threadIdx.x == 0) s_pos0 = pos;
    __syncthreads();
    const bool fits = k >= N || (ok && pos == s_pos0 + rel);
    if (__syncthreads_and(fits)) {
      if (ok) {
        for (uint32_t j = 0; j < L; ++j) {
          const uint32_t b = sh + j;
          s_txt[rel + j] = (uint8_t)(wv[b >> 2] >> (8 * (b & 3)));
        }
        if (s) s_txt[rel + L] = (uint8_t)sep;
      }
      __syncthreads();
      lds_bytes_to_global<NT>(s_txt, total, out + s_pos0);
    } else if (ok) {
      for (uint32_t j = 0; j < L; ++j) {
        const uint32_t b = sh + j;
        out[pos + j] = (uint8_t)(wv[b >> 2] >> (8 * (b & 3)));
      }
      if (s) out[pos + L] = (uint8_t)sep;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- k_keys_text
// Sorted text from the sorted keys, in the same run as the sort.  A word is
// at most 32 bytes, so its key lanes (big-endian, zero padded) hold all of its
// bytes; when the run asks for text, every segment's chunk sort or last merge
// level leaves its sorted keys in a key buffer besides writing the indices:
// buffer A when the segment took an even number of merge passes (none
// included), B when odd.  So the text is written from keys read in order, and
// no word is read again from the input at a random place.
//
// Positions of the sorted order (documents in turn, each document's lengths
// in turn: the order of the output permutation) are cut into tiles of W; a
// workgroup takes a contiguous range of tiles.  For a batch of up to NT
// tiles, thread k first finds where tile k starts: its (document, length)
// segment and its first byte in the text.  Then tile by tile the workgroup
// cuts the tile into the pieces of the segments it covers, assembles the
// text of its words in LDS -- each word followed by the separator when there
// is one, laid out on the output's dword grid, the dwords wholly inside a
// word written whole and only its edges by byte and halfword -- and stores
// it as one stretch (a tile whose text outgrows the LDS stretch, KTB bytes per word
// on average, writes its words straight to memory instead).  The layout is
// the permutation-based writer's: document d's text
// starts at byte (offsets[first word of d] - offsets[0]) + (first word of d)
// when words are separated, without the second term otherwise.
struct TextAt {
  uint32_t seg;   // (document, length) segment holding the position
  uint64_t pos;   // the position's first text byte
};

// Segment and text byte of sorted position g (g < N).  Empty documents and
// segments start where the next one does, so "the last one starting at or
// before g" skips them.
__device__ inline TextAt text_at(const Ws& w, const RunDesc& d, uint32_t D, uint32_t sw, uint32_t g) {
  uint32_t lo = 0, hi = D;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (w.doc_off[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  const uint32_t* sb = w.seg_base + (size_t)lo * kNB;
  uint32_t L = 0;
#pragma unroll
  for (uint32_t step = 32; step >= 1; step >>= 1)
    if (L + step <= (uint32_t)kMaxLen && sb[L + step] <= g) L += step;
  const uint32_t f = w.doc_off[lo];
  uint64_t pos = (uint64_t)(d.offsets[f] - d.offsets[0]) + (uint64_t)sw * f;
  const uint32_t* sn = w.seg_n + (size_t)lo * kNB;
#pragma unroll
  for (uint32_t l = 0; l < (uint32_t)kMaxLen; ++l)
    if (l < L) pos += (uint64_t)sn[l] * (l + sw);
  return TextAt{lo * kNB + L, pos + (uint64_t)(g - sb[L]) * (L + sw)};
}

constexpr uint32_t kTextDwordMin = 12;   // words of this many text bytes or more are written by dwords

// The L bytes of a word from its big-endian key lanes, then the separator
// when there is one (sw = 1), one byte at a time: for short words, whose
// dword writer would mostly make partial stores at both edges.  Called with
// an LDS or a global destination, so that each gets its own stores.
template <class P>
__device__ inline void put_word_bytes(P dst, const uint64_t (&ln)[4], uint32_t L, uint32_t sw, uint8_t sep) {
  uint64_t cur = ln[0];
  for (uint32_t j = 0; j < L; ++j) {
    dst[j] = (uint8_t)(cur >> 56);
    cur <<= 8;
    if ((j & 7u) == 7u) cur = j == 7u ? ln[1] : (j == 15u ? ln[2] : ln[3]);
  }
  if (sw) dst[L] = sep;
}

template <int NT, int IPT, int KTB>
__global__ __launch_bounds__(NT) void k_keys_text(Ws w) {
  constexpr uint32_t W = NT * IPT;
  constexpr uint32_t CAP = W * KTB;      // LDS text bytes of a tile
  static_assert(NT < 1024 && W * (kMaxLen + 1) < (1u << 22), "piece count and text bytes share one scan");
  static_assert(W < 65536, "tile positions are 16-bit");
  __shared__ uint32_t s_txt32[CAP / 4 + 2];
  __shared__ uint16_t s_first[W + 1];   // first tile position of each piece
  __shared__ uint32_t s_rel[W];         // its first text byte, counted from the dword below the tile's first
  __shared__ uint16_t s_info[W];        // length, plus 256 when its keys are in buffer B
  __shared__ uint32_t s_tseg[NT + 1];   // per tile of the batch: segment of its first position
  __shared__ uint64_t s_tpos[NT + 1];   // ... and that position's first text byte
  __shared__ uint32_t s_tmp[NT / 64];
  uint8_t* s_txt = (uint8_t*)s_txt32;
  Header* h = w.h;
  if (h->abort) return;
  const RunDesc d = h->d;
  if (d.out_text == nullptr) return;
  const uint32_t N = h->n_words, D = h->n_docs;
  const uint32_t sw = d.sep >= 0 ? 1u : 0u;
  const uint64_t out_size = (uint64_t)(d.offsets[N] - d.offsets[0]) + (uint64_t)sw * N;
  const uint32_t ntiles = (N + W - 1) / W;
  const uint32_t G = gridDim.x, q = ntiles / G, rem = ntiles % G;
  const uint32_t nb = q + (blockIdx.x < rem ? 1u : 0u);
  const uint32_t tb = blockIdx.x * q + min(blockIdx.x, rem);
  for (uint32_t c0 = 0; c0 < nb; c0 += NT) {
    const uint32_t cn = min((uint32_t)NT, nb - c0);
    // where tiles tb+c0 .. tb+c0+cn-1 start, and the segment of the last
    // position of the batch (bounding the last tile's pieces)
    for (uint32_t k = threadIdx.x; k <= cn; k += NT) {
      const uint32_t g = min((tb + c0 + k) * W, N - 1);
      const TextAt at = text_at(w, d, D, sw, g);
      s_tseg[k] = at.seg;
      s_tpos[k] = at.pos;
    }
    __syncthreads();
    for (uint32_t k = 0; k < cn; ++k) {
      const uint32_t t = tb + c0 + k;
      const uint32_t g0 = t * W, g1 = min(N, g0 + W);
      const uint32_t S0 = s_tseg[k], S1 = s_tseg[k + 1];
      const uint64_t pos0 = s_tpos[k];
      // LDS byte of the tile's first text byte: its place in the output's dword grid
      const uint32_t head = (uint32_t)(((uintptr_t)d.out_text + pos0) & 3u);
      // the pieces: segments S0..S1 clipped to [g0, g1), the empty ones
      // dropped; one scan counts them (low 10 bits) and their text bytes
      uint32_t npieces = 0, tbytes = 0;
      for (uint32_t sbase = S0; sbase <= S1; sbase += NT) {
        const uint32_t sg = sbase + threadIdx.x;
        const uint32_t L = sg % kNB;
        uint32_t cnt = 0, first = 0, info = 0;
        if (sg <= S1) {
          const uint32_t b = w.seg_base[sg], n = w.seg_n[sg];
          const uint32_t a = max(b, g0), e = min(b + n, g1);
          if (e > a) {
            cnt = e - a;
            first = a - g0;
            const int c = class_of_len(L);
            const uint32_t m = n <= kPackMax ? 0u : merge_passes(n, w.T[c], w.fan[c]);
            info = L | ((m & 1u) << 8);
          }
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<NT>((cnt ? 1u : 0u) | ((cnt * (L + sw)) << 10), s_tmp, tot);
        if (cnt) {
          s_first[npieces + (ex & 1023u)] = (uint16_t)first;
          s_rel[npieces + (ex & 1023u)] = head + tbytes + (ex >> 10);
          s_info[npieces + (ex & 1023u)] = (uint16_t)info;
        }
        npieces += tot & 1023u;
        tbytes += tot >> 10;
      }
      if (threadIdx.x == 0) s_first[npieces] = (uint16_t)(g1 - g0);
      __syncthreads();
      if (pos0 + tbytes > out_size) {   // cannot happen for checked offsets; never write past the text
        if (threadIdx.x == 0) atomicOr(&h->status, ST_INVALID);
        continue;
      }
      const bool staged = head + tbytes <= CAP;
      uint8_t* out = d.out_text + pos0 - head;   // dword aligned; byte `head` is the tile's first
      // every word's key lanes are requested before any is used
      uint64_t ln[IPT][4];
      uint32_t wl[IPT], wrel[IPT];
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t i = threadIdx.x + (uint32_t)r * NT;
        wl[r] = 0;
        wrel[r] = 0;
        ln[r][0] = ln[r][1] = ln[r][2] = ln[r][3] = 0;
        if (g0 + i < g1) {
          uint32_t lo = 0, hi = npieces;   // the last piece starting at or before i
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_first[mid] <= i)
              lo = mid;
            else
              hi = mid;
          }
          const uint32_t info = s_info[lo], L = info & 255u;
          const bool inb = (info >> 8) != 0;
          const size_t g = (size_t)g0 + i;
          wl[r] = L;
          wrel[r] = s_rel[lo] + (i - s_first[lo]) * (L + sw);
          ln[r][0] = (inb ? w.b.k[0] : w.a.k[0])[g];   // class 0: its index in the low half is masked off
          if (L > 8) ln[r][1] = (inb ? w.b.k[1] : w.a.k[1])[g];
          if (L > 16) ln[r][2] = (inb ? w.b.k[2] : w.a.k[2])[g];
          if (L > 24) ln[r][3] = (inb ? w.b.k[3] : w.a.k[3])[g];
        }
      }
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t L = wl[r], rel = wrel[r];
        if (threadIdx.x + (uint32_t)r * NT < g1 - g0) {
          const bool dw = L + sw >= kTextDwordMin;
          if (staged && dw)
            put_word_text(s_txt + (rel & ~3u), rel & 3u, ln[r], L, sw, (uint32_t)d.sep);
          else if (staged)
            put_word_bytes(s_txt + rel, ln[r], L, sw, (uint8_t)d.sep);
          else if (dw)
            put_word_text(out + (rel & ~3u), rel & 3u, ln[r], L, sw, (uint32_t)d.sep);
          else
            put_word_bytes(out + rel, ln[r], L, sw, (uint8_t)d.sep);
        }
      }
      __syncthreads();
      if (staged) {
        // LDS byte j holds the output byte at out + j
        const uint32_t e = head + tbytes;
        const uint32_t fb = min(e, 4u);                  // bytes of the first dword
        const uint32_t nd = e > 4 ? (e - 4) / 4 : 0u;    // whole dwords after it
        for (uint32_t j = head + threadIdx.x; j < fb; j += NT) out[j] = s_txt[j];
        uint32_t* o32 = (uint32_t*)(out + 4);
        for (uint32_t j = threadIdx.x; j < nd; j += NT) o32[j] = s_txt32[1 + j];
        for (uint32_t j = 4 + 4 * nd + threadIdx.x; j < e; j += NT) out[j] = s_txt[j];
      }
      __syncthreads();
    }
  }
}

}  // namespace sw
