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
// output positions.
#pragma once

#include "sw_device.hpp"

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

__device__ inline bool tok_space(uint32_t c) { return c == 32u || (c - 9u) < 5u; }
__device__ inline bool tok_letter(uint32_t c) { return ((c | 32u) - 97u) < 26u; }

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

__device__ inline TokSum tok_summary(const uint32_t (&w)[16]) {
  TokSum s{0, 0, 0, TS_NONE};
  uint32_t cur = TS_NONE;
  bool first_open = false;   // a letter met while the incoming state was still unknown
#pragma unroll
  for (int b = 0; b < kTokBytes; ++b) {
    const uint32_t c = (w[b >> 2] >> (8 * (b & 3))) & 0xFFu;
    if (tok_space(c)) {
      cur = TS_SPACE;
    } else if (tok_letter(c)) {
      s.letters += 1;
      if (cur == TS_SPACE) s.starts_letter += 1;
      if (cur == TS_NONE) first_open = true;
      cur = TS_LETTER;
    }
  }
  s.starts_space = s.starts_letter + (first_open ? 1u : 0u);
  s.last = cur;
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
  const TokSum s = tok_summary(w);
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
// grid, so that the stretch is stored as whole dwords); the offsets of the
// words that start among them go straight to memory (a thread's words are
// consecutive there).
__global__ __launch_bounds__(kTokNT) void k_tok_write(Header* h, const uint8_t* text, uint64_t n, const uint4* pre,
                                                      uint32_t flags, uint8_t* out_chars, uint32_t* out_offsets) {
  __shared__ uint32_t s_last[kTokNT / 64];
  __shared__ uint32_t s_tmp[kTokNT / 64];
  __shared__ uint32_t s_chr32[kTokBlock / 4 + 2];
  if (h->abort) return;
  uint8_t* s_chr = (uint8_t*)s_chr32;
  const uint64_t b = blockIdx.x;
  const uint64_t p = b * kTokBlock + (uint64_t)threadIdx.x * kTokBytes;
  const uint32_t cnt = p < n ? (uint32_t)min<uint64_t>(kTokBytes, n - p) : 0u;
  uint32_t w[16];
  tok_load(text, p, cnt, w);
  const TokSum s = tok_summary(w);
  const uint4 bp = pre[b];
  uint32_t carry = tok_carry_in_block<kTokNT>(s.last, s_last);
  if (carry == TS_NONE) carry = bp.z;
  const uint32_t starts = carry == TS_LETTER ? s.starts_letter : s.starts_space;
  uint32_t nl, nwd;
  const uint32_t lrel = block_excl_scan<kTokNT>(s.letters, s_tmp, nl);   // inside the workgroup
  uint32_t wpos = bp.y + block_excl_scan<kTokNT>(starts, s_tmp, nwd);
  const uint32_t head = (uint32_t)((uintptr_t)(out_chars + bp.x) & 3u);   // LDS byte of the stretch's first letter
  const uint32_t fold = (flags & kTokFlagLower) ? 32u : 0u;
  uint32_t lpos = lrel;
  uint32_t cur = carry;
  for (uint32_t i = 0; i < cnt; ++i) {
    const uint32_t c = (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
    if (tok_space(c)) {
      cur = TS_SPACE;
    } else if (tok_letter(c)) {
      if (cur != TS_LETTER) out_offsets[wpos++] = bp.x + lpos;
      s_chr[head + lpos++] = (uint8_t)(c | (c < 97u ? fold : 0u));
      cur = TS_LETTER;
    }
  }
  __syncthreads();
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

}  // namespace sw
