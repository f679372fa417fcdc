// sw_kernels.hpp -- HIP kernels of the gfx950 word sort.
//
// One pass (arXiv:1411.5283, section 3 "Pre-processing" phases 2-3, sections
// 3.2 and 4 for the chunked parallel form):
//   k_begin        run descriptor into the workspace, status cleared
//   k_doc_plan     documents -> word blocks (a block never spans documents)
//   k_hist         per-block length histogram; offsets validated
//   k_scan_rows    prefix of the histogram over blocks, per length
//   k_segments     per (document, length) segment: size and first position;
//                  the document's bucket offsets
//   k_seg_count / k_scan_rows / k_seg_scatter
//                  segments ordered by (key class, merge levels descending) so
//                  that the segments still merging at level l are a prefix
//   k_tile_prefix  per class: tiles of the chunk sort and of a two-way merge
//                  level, words of the four-way merge's ranges
//   k_scatter_pack stable distribution of the words into their segment, as
//                  big-endian key lanes + index (the sub-arrays of phase 2)
//   k_sort_tiles   per tile: odd-even transposition on chunks (bubble sort's
//                  parallel form), then merge-path merges in LDS up to the tile
//   k_merge        one two-way merge-path level over HBM (each workgroup
//                  places its own tiles); the last level of a segment writes
//                  the output permutation
//   k_merge4w      one four-way merge pass over HBM (two doublings of the
//                  run length per pass, in steps of bounded windows)
//   k_pack_full    the same words as one sequence of full keys (baseline
//                  without length lists)
// Every kernel after k_begin reads the run from the workspace, so the same
// sequence runs eagerly or as one captured HIP graph.
#pragma once
#include "sw_device.hpp"
#include "sw_split.hpp"
#include "sw_window.hpp"

namespace sw {


// ---------------------------------------------------------------- k_begin
__global__ void k_begin(Ws w, RunDesc d) {
  if (threadIdx.x == 0) {
    Header* h = w.h;
    h->d = d;
    h->status = 0;
    h->abort = 0;
    h->n_docs = d.doc_offsets ? d.n_docs : 1u;
    h->n_words = 0;
    h->n_blocks = 0;
    h->n_segs = 0;
    h->n_segblocks = 0;
  }
}

// The run's status word, copied out for a caller that has no access to the
// workspace.
__global__ void k_status_out(Ws w, uint32_t* dst) {
  if (threadIdx.x == 0) *dst = w.h->status;
}

// ---------------------------------------------------------------- k_doc_plan
// One workgroup.  Copies (or synthesizes) the document offsets, validates
// them, and gives every document ceil(words / kWordsPerBlock) word blocks.
template <int NT>
__global__ __launch_bounds__(NT) void k_doc_plan(Ws w) {
  __shared__ uint32_t s_tmp[NT / 64];
  __shared__ uint32_t s_bad;
  Header* h = w.h;
  const RunDesc d = h->d;
  const uint32_t D = h->n_docs;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  uint32_t carry = 0;
  uint32_t bad = 0;
  for (uint32_t base = 0; base <= D; base += NT) {
    const uint32_t j = base + threadIdx.x;
    uint32_t nb = 0;
    if (j <= D) {
      const uint32_t s = d.doc_offsets ? d.doc_offsets[j] : (j == 0 ? 0u : d.n_words);
      w.doc_off[j] = s;
      if (j == 0 && s != 0) bad |= ST_INVALID;
      if (j > 0) {
        const uint32_t prev = d.doc_offsets ? d.doc_offsets[j - 1] : 0u;
        if (s < prev)
          bad |= ST_INVALID;
        else
          nb = (s - prev + kWordsPerBlock - 1) / kWordsPerBlock;
      }
      if (j == D && s > w.Nmax) bad |= ST_WORKSPACE;
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan<NT>(nb, s_tmp, total);
    if (j <= D) w.doc_blk[j] = carry + ex + nb;   // blocks of documents 0..j-1
    carry += total;
  }
  if (bad) atomicOr(&s_bad, bad);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_bad) {
      atomicOr(&h->status, s_bad);
      atomicOr(&h->abort, 1u);
    } else {
      h->n_words = w.doc_off[D];
      h->n_blocks = carry;
      h->n_segs = D * (uint32_t)kNB;
      h->n_segblocks = (D * (uint32_t)kNB + kSegsPerBlock - 1) / kSegsPerBlock;
    }
  }
}

// Word range of word block b: its document and [ws, we).
struct BlockRange {
  uint32_t doc, ws, we;
};
template <int NT>
__device__ inline BlockRange block_range(const Ws& w, uint32_t b, uint32_t D, uint32_t* s_doc) {
  if (threadIdx.x < 64) {
    const uint32_t dd = wave_find(w.doc_blk, D + 1, b);
    if (threadIdx.x == 0) *s_doc = dd;
  }
  __syncthreads();
  BlockRange r;
  r.doc = *s_doc;
  r.ws = w.doc_off[r.doc] + (b - w.doc_blk[r.doc]) * kWordsPerBlock;
  r.we = min(r.ws + kWordsPerBlock, w.doc_off[r.doc + 1]);
  return r;
}

// ---------------------------------------------------------------- k_hist
// Length histogram per word block (phase 2: sub-array sizes are the counts
// of words of each length).  Also validates the offsets.
template <int NT>
__global__ __launch_bounds__(NT) void k_hist(Ws w) {
  __shared__ uint32_t s_cnt[kNB];
  __shared__ uint32_t s_doc;
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t nblk = h->n_blocks;
  const uint32_t D = h->n_docs;
  const uint32_t N = h->n_words;
  const uint32_t* off = h->d.offsets;
  const bool no_chars = h->d.chars == nullptr;
  const uint32_t off_lo = off[0], off_hi = off[N];
  const uint32_t rs = w.Bmax + 1;
  uint32_t flags = 0;
  // the characters must fit the capacity the workspace was made for
  if (blockIdx.x == 0 && off_hi >= off_lo && (uint64_t)(off_hi - off_lo) > w.Cmax) flags |= ST_WORKSPACE;
  for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    if (threadIdx.x < kNB) s_cnt[threadIdx.x] = 0;
    const BlockRange r = block_range<NT>(w, b, D, &s_doc);   // has a barrier
    // all of this thread's offsets are requested before any is used, so the
    // block waits for one memory latency, not one per word
    constexpr int IT = kWordsPerBlock / NT;
    uint32_t oa[IT], oe[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t i = r.ws + threadIdx.x + k * NT;
      oa[k] = i < r.we ? off[i] : 0u;
      oe[k] = i < r.we ? off[i + 1] : 0u;
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t i = r.ws + threadIdx.x + k * NT;
      if (i < r.we) {
        const uint32_t a = oa[k], e = oe[k];
        uint32_t L = e - a;
        if (e < a || a < off_lo || e > off_hi || (no_chars && e != a)) {
          flags |= ST_INVALID;
          L = 0;
        } else if (L > (uint32_t)kMaxLen) {
          flags |= ST_TOO_LONG;
          L = kMaxLen;
        }
        atomicAdd(&s_cnt[L], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x < kNB) w.cnt[threadIdx.x * rs + b] = s_cnt[threadIdx.x];
    __syncthreads();
  }
  if (__any(flags != 0)) {
    // one atomic per wave
    uint32_t f = flags;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) f |= __shfl_xor(f, o);
    if (__lane_id() == 0 && f) {
      atomicOr(&h->status, f);
      atomicOr(&h->abort, 1u);
    }
  }
}

// ---------------------------------------------------------------- k_scan_rows
// Exclusive prefix of each row over its first *ncols entries; the row total
// goes to entry *ncols.  One workgroup per row (grid-stride over rows).
template <int NT, int IPT>
__global__ __launch_bounds__(NT) void k_scan_rows(Ws w, uint32_t* rows, uint32_t nrows,
                                                   uint32_t stride, int which) {
  __shared__ uint32_t s_tmp[NT / 64];
  const Header* h = w.h;
  if (h->abort) return;
  const uint32_t ncols = which == 0 ? h->n_blocks : h->n_segblocks;
  for (uint32_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    uint32_t* row = rows + (size_t)r * stride;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < ncols; base += NT * IPT) {
      uint32_t v[IPT];
      uint32_t sum = 0;
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const uint32_t i = base + threadIdx.x * IPT + k;
        v[k] = i < ncols ? row[i] : 0u;
        sum += v[k];
      }
      uint32_t total;
      uint32_t run = carry + block_excl_scan<NT>(sum, s_tmp, total);
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const uint32_t i = base + threadIdx.x * IPT + k;
        if (i < ncols) row[i] = run;
        run += v[k];
      }
      carry += total;
    }
    if (threadIdx.x == 0) row[ncols] = carry;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- k_segments
// One wave per document: counts of its 33 lengths, their exclusive prefix
// (the document's bucket offsets, an output), and the segment table.
template <int NT>
__global__ __launch_bounds__(NT) void k_segments(Ws w) {
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t D = h->n_docs;
  const uint32_t rs = w.Bmax + 1;
  const uint32_t lane = __lane_id();
  const uint32_t waves = gridDim.x * (NT / 64);
  uint32_t* out_boff = h->d.out_boff;
  for (uint32_t dd = blockIdx.x * (NT / 64) + (threadIdx.x >> 6); dd < D; dd += waves) {
    const uint32_t b0 = w.doc_blk[dd], b1 = w.doc_blk[dd + 1];
    const uint32_t c = lane < (uint32_t)kNB ? w.cnt[lane * rs + b1] - w.cnt[lane * rs + b0] : 0u;
    const uint32_t ex = wave_incl_scan(c) - c;
    if (lane < (uint32_t)kNOff) out_boff[(size_t)dd * kNOff + lane] = ex;
    if (lane < (uint32_t)kNB) {
      w.seg_n[dd * kNB + lane] = c;
      w.seg_base[dd * kNB + lane] = w.doc_off[dd] + ex;
    }
  }
}

// Segment order key: class, then merge levels descending, then the short
// segments that are packed several to a tile; empty segments last.
__device__ inline uint32_t seg_key(const Ws& w, uint32_t s) {
  const uint32_t n = w.seg_n[s];
  if (n == 0) return kNKeys - 1;
  const int c = class_of_len(s % kNB);
  if (n <= kPackMax) return (uint32_t)c * kMaxLev + (kMaxLev - 1);
  const uint32_t m = levels_for(n, w.T[c]);
  return (uint32_t)c * kMaxLev + (kMaxLev - 2 - m);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_seg_count(Ws w) {
  __shared__ uint32_t s_cnt[kNKeys];
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t S = h->n_segs, nsb = h->n_segblocks;
  const uint32_t rs = w.SBmax + 1;
  for (uint32_t b = blockIdx.x; b < nsb; b += gridDim.x) {
    for (uint32_t k = threadIdx.x; k < (uint32_t)kNKeys; k += NT) s_cnt[k] = 0;
    __syncthreads();
    const uint32_t lo = b * kSegsPerBlock, hi = min(S, lo + kSegsPerBlock);
    for (uint32_t s = lo + threadIdx.x; s < hi; s += NT) atomicAdd(&s_cnt[seg_key(w, s)], 1u);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < (uint32_t)kNKeys; k += NT) w.segcnt[k * rs + b] = s_cnt[k];
    __syncthreads();
  }
}

// Stable counting-sort scatter of the segments by seg_key.  Each wave ranks a
// contiguous quarter of the block: lanes with equal keys are found with
// ballots, a per-wave running count carries ranks across iterations.
template <int NT>
__global__ __launch_bounds__(NT) void k_seg_scatter(Ws w) {
  constexpr int NW = NT / 64;
  constexpr uint32_t PER_WAVE = kSegsPerBlock / NW;
  constexpr int IT = PER_WAVE / 64;
  __shared__ uint32_t s_run[NW][kNKeys];
  __shared__ uint32_t s_kbase[kNKeys];
  __shared__ uint32_t s_tmp[NW];
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t S = h->n_segs, nsb = h->n_segblocks;
  const uint32_t rs = w.SBmax + 1;
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  {
    const uint32_t tot = threadIdx.x < (uint32_t)kNKeys ? w.segcnt[threadIdx.x * rs + nsb] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<NT>(tot, s_tmp, total);
    if (threadIdx.x < (uint32_t)kNKeys) s_kbase[threadIdx.x] = ex;
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x <= (uint32_t)kNClass) h->cls_start[threadIdx.x] = s_kbase[threadIdx.x * kMaxLev];
    if (threadIdx.x < (uint32_t)kNClass) h->pack_start[threadIdx.x] = s_kbase[threadIdx.x * kMaxLev + kMaxLev - 1];
    for (uint32_t i = threadIdx.x; i < (uint32_t)(kNClass * kMaxLev); i += NT) {
      const uint32_t c = i / kMaxLev, l = i % kMaxLev;
      h->active[c][l] = l + 2 <= (uint32_t)kMaxLev
                            ? s_kbase[c * kMaxLev + (kMaxLev - 2 - l)] - s_kbase[c * kMaxLev]
                            : 0u;
    }
  }
  for (uint32_t b = blockIdx.x; b < nsb; b += gridDim.x) {
    for (uint32_t k = threadIdx.x; k < (uint32_t)(NW * kNKeys); k += NT) (&s_run[0][0])[k] = 0;
    __syncthreads();
    const uint32_t wbeg = b * kSegsPerBlock + wave * PER_WAVE;
    uint32_t pk[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const uint32_t s = wbeg + it * 64 + lane;
      const bool valid = s < S;
      const uint32_t key = valid ? seg_key(w, s) : 0u;
      const uint64_t mm = match_mask<kKeyBits>(key, valid);
      const uint32_t r = lanes_below(mm);
      const uint32_t old = valid ? s_run[wave][key] : 0u;
      if (valid && r == 0) s_run[wave][key] = old + (uint32_t)__popcll(mm);
      pk[it] = key | ((old + r) << kKeyBits);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < (uint32_t)kNKeys; k += NT) {
      uint32_t acc = 0;
      for (int v = 0; v < NW; ++v) {
        const uint32_t t = s_run[v][k];
        s_run[v][k] = acc;
        acc += t;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const uint32_t s = wbeg + it * 64 + lane;
      const uint32_t key = pk[it] & ((1u << kKeyBits) - 1);
      if (s < S && key != (uint32_t)(kNKeys - 1)) {
        const uint32_t dest = s_kbase[key] + w.segcnt[key * rs + b] + s_run[wave][key] + (pk[it] >> kKeyBits);
        w.sorted[dest] = s;
      }
    }
    __syncthreads();
  }
}

// Per class (blockIdx.x / 4) and kind (blockIdx.x % 4): exclusive prefix over
// the class sublist of the chunk-sort tiles (kind 0), the two-way merge tiles
// (kind 1) or the words (kind 3, the four-way merge's ranges) of its segments
// that are not packed, or of the sizes of its short segments (kind 2, their
// positions in the packed tiles).
template <int NT>
__global__ __launch_bounds__(NT) void k_tile_prefix(Ws w) {
  __shared__ uint32_t s_tmp[NT / 64];
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t c = blockIdx.x / 4, kind = blockIdx.x % 4;
  const uint32_t cs = kind == 2 ? h->pack_start[c] : h->cls_start[c];
  const uint32_t ce = kind == 2 ? h->cls_start[c + 1] : h->pack_start[c];
  uint32_t* out = (kind == 0 ? w.st : (kind == 1 ? w.mt : (kind == 2 ? w.vpre : w.wpre))) +
                  (kind == 2 ? cs : h->cls_start[c]) + c;
  const uint32_t div = kind == 0 ? w.T[c] : (kind == 1 ? w.P[c] : 1u);
  uint32_t carry = 0;
  for (uint32_t base = cs; base < ce; base += NT) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < ce ? (w.seg_n[w.sorted[i]] + div - 1) / div : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<NT>(v, s_tmp, total);
    if (i < ce) out[i - cs] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    out[ce - cs] = carry;
    if (kind == 0) h->sort_tiles[c] = carry;
    if (kind == 2) h->pack_words[c] = carry;
  }
}

// ---------------------------------------------------------------- packing
// Big-endian lanes of the L-byte word at p, zero padded.  Reads only the
// aligned dwords that hold at least one byte of the word.
template <int NQ>
__device__ inline void load_be_lanes(const uint8_t* p, uint32_t L, uint64_t (&lane)[NQ]) {
  const uintptr_t addr = (uintptr_t)p;
  const uint32_t* base = (const uint32_t*)(addr & ~(uintptr_t)3);
  const uint32_t s = (uint32_t)(addr & 3);
  const uint32_t nd = L ? (s + L + 3) >> 2 : 0u;
  uint32_t wv[2 * NQ + 1];
#pragma unroll
  for (int j = 0; j < 2 * NQ + 1; ++j) wv[j] = (uint32_t)j < nd ? __builtin_bswap32(base[j]) : 0u;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const uint64_t hi = ((uint64_t)wv[2 * q] << 32) | wv[2 * q + 1];
    uint64_t v = s ? (hi << (8 * s)) | (uint64_t)(wv[2 * q + 2] >> (32 - 8 * s)) : hi;
    const int rem = (int)L - 8 * q;
    v = rem >= 8 ? v : (rem <= 0 ? 0ull : (v & (~0ull << (64 - 8 * rem))));
    lane[q] = v;
  }
}

// Big-endian bytes of a word staged in LDS as dwords d[0], d[1], ... with its
// first byte at byte s (0..3) of d[0].  Bytes 4t..4t+3 of the word are bytes
// s..s+3 of the eight-byte pair (d[t+1]:d[t]); v_perm picks them most
// significant first with the selector s*0x01010101 + 0x00010203, and a
// selector byte of 0x0C yields a zero byte.
__device__ inline uint32_t be_sel(uint32_t s) { return s * 0x01010101u + 0x00010203u; }
__device__ inline uint32_t be_word(const uint32_t* d, int t, uint32_t sel) {
  return __builtin_amdgcn_perm(d[t + 1], d[t], sel);
}

// Lanes of a class-C word of length L (C >= 1: 8(C-1) < L <= 8C) from LDS:
// lanes 0..C-2 are full; the last keeps its first L - 8(C-1) bytes.
template <int C>
__device__ inline void lds_class_lanes(const uint32_t* d, uint32_t s, uint32_t L, uint64_t (&lane)[C]) {
  const uint32_t sel = be_sel(s);
#pragma unroll
  for (int q = 0; q < C; ++q) lane[q] = ((uint64_t)be_word(d, 2 * q, sel) << 32) | be_word(d, 2 * q + 1, sel);
  lane[C - 1] &= ~0ull << (64 * C - 8 * L);
}

// ---------------------------------------------------------------- k_scatter_pack
// Stable scatter of every word into its (document, length) segment, packed
// into key lanes.  The block's offsets, and its characters when they fit
// kScatterChars bytes, are first staged in LDS with 16-byte loads from
// 16-byte aligned addresses (the few words before the block's first offset or
// character in its 16 bytes come along and are skipped).
// Pass 1: the rank of a word among the words of the same length before it in
// the block (per wave with ballots, a running count per wave carries ranks
// across iterations) gives its slot in the block's length-sorted order; LDS
// records which word holds each slot.  Pass 2 walks the slots in order, class
// by class (a class's slots are contiguous), so consecutive lanes write
// consecutive positions of one segment (coalesced stores) and build the lanes
// of one class, reading the words from LDS.
constexpr uint32_t kScatterChars = 24576;   // three workgroups per CU; a block of 4096 words averages about 18 KB

template <int NW>
struct ScatterLds {
  uint4 off4[(kWordsPerBlock + 1 + 3 + 3) / 4];   // the block's offsets after up to 3 dwords of lead
  uint4 chr4[kScatterChars / 16 + 2];              // + the dwords a word's lanes may read past the end
  uint16_t slot[kWordsPerBlock];
  uint32_t run[NW][kNB];
  uint32_t bstart[kNB + 1];
  uint32_t dst[kNB];     // segment position of slot 0 of each length
  uint32_t doc;
};

// Pass 2 for the slots [ps, pe) of class C.
template <int NT, int C>
__device__ inline void scatter_class(const Ws& w, const ScatterLds<NT / 64>& S, const uint32_t* s_off, uint32_t ps,
                                     uint32_t pe, bool staged, uint32_t cpos, uint32_t ibase,
                                     const uint8_t* chars) {
  const uint32_t* s_chr = (const uint32_t*)S.chr4;
  for (uint32_t p = ps + threadIdx.x; p < pe; p += NT) {
    const uint32_t i = S.slot[p];
    const uint32_t a = s_off[i];
    const uint32_t L = min(s_off[i + 1] - a, (uint32_t)kMaxLen);
    const uint32_t dest = S.dst[L] + p;
    const uint32_t idx = ibase + i;
    if constexpr (C == 0) {
      uint64_t hi;
      if (staged) {
        const uint32_t pos = a + cpos;
        // the word's L (0..4) bytes: selector bytes past them become 0x0C
        const uint32_t keep = (uint32_t)(0xFFFFFFFF00000000ull >> (8 * L));
        const uint32_t sel = (be_sel(pos & 3) & keep) | (0x0C0C0C0Cu & ~keep);
        hi = (uint64_t)be_word(s_chr + (pos >> 2), 0, sel) << 32;
      } else {
        uint64_t ln[1];
        load_be_lanes<1>(chars + a, L, ln);
        hi = ln[0] & 0xFFFFFFFF00000000ull;
      }
      w.a.k[0][dest] = hi | idx;
    } else {
      uint64_t ln[C];
      if (staged) {
        const uint32_t pos = a + cpos;
        lds_class_lanes<C>(s_chr + (pos >> 2), pos & 3, L, ln);
      } else {
        load_be_lanes<C>(chars + a, L, ln);
      }
#pragma unroll
      for (int q = 0; q < C; ++q) w.a.k[q][dest] = ln[q];
      w.a.idx[dest] = idx;
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_scatter_pack(Ws w) {
  constexpr int NW = NT / 64;
  constexpr uint32_t PER_WAVE = kWordsPerBlock / NW;
  constexpr int IT = PER_WAVE / 64;
  static_assert(kWordsPerBlock <= 65536, "slot index is 16-bit");
  __shared__ ScatterLds<NW> S;
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t nblk = h->n_blocks, D = h->n_docs;
  const uint32_t* off = h->d.offsets;
  const uint8_t* chars = h->d.chars;
  const uint32_t rs = w.Bmax + 1;
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    for (uint32_t k = threadIdx.x; k < (uint32_t)(NW * kNB); k += NT) (&S.run[0][0])[k] = 0;
    const BlockRange r = block_range<NT>(w, b, D, &S.doc);   // has a barrier
    const uint32_t nw = r.we - r.ws;
    // offsets [ws, we] and characters [off[ws], off[we]) as whole aligned
    // 16-byte pieces; olead dwords and lead bytes precede the block's own
    const uintptr_t oaddr = (uintptr_t)(off + r.ws);
    const uint4* osrc = (const uint4*)(oaddr & ~(uintptr_t)15);
    const uint32_t olead = (uint32_t)(oaddr & 15) >> 2;
    const uint32_t n_o4 = (olead + nw + 1 + 3) >> 2;
    const uint32_t c0 = off[r.ws], c1 = off[r.we];
    const uintptr_t caddr = (uintptr_t)(chars + c0);
    const uint4* csrc = (const uint4*)(caddr & ~(uintptr_t)15);
    const uint32_t lead = (uint32_t)(caddr & 15);
    const uint32_t n_c4 = c1 > c0 ? (lead + (c1 - c0) + 15) >> 4 : 0u;
    const bool staged = n_c4 <= kScatterChars / 16;
    {
      constexpr int UNR = 4;
      const uint32_t ntot = n_o4 + (staged ? n_c4 : 0u);
      for (uint32_t k0 = 0; k0 < ntot; k0 += NT * UNR) {
        uint4 v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const uint32_t k = k0 + threadIdx.x + u * NT;
          v[u] = k < ntot ? (k < n_o4 ? osrc[k] : csrc[k - n_o4]) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const uint32_t k = k0 + threadIdx.x + u * NT;
          if (k < n_o4)
            S.off4[k] = v[u];
          else if (k < ntot)
            S.chr4[k - n_o4] = v[u];
        }
      }
    }
    const uint32_t* s_off = (const uint32_t*)S.off4 + olead;
    if (threadIdx.x < (uint32_t)kNB) {
      const uint32_t L = threadIdx.x;
      S.dst[L] = w.seg_base[r.doc * kNB + L] + w.cnt[L * rs + b] - w.cnt[L * rs + w.doc_blk[r.doc]];
    }
    __syncthreads();
    const uint32_t wofs = wave * PER_WAVE;
    uint32_t pk[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const uint32_t i = wofs + it * 64 + lane;      // word index inside the block
      const bool valid = i < nw;
      uint32_t L = 0;
      if (valid) L = min(s_off[i + 1] - s_off[i], (uint32_t)kMaxLen);
      const uint64_t mm = match_mask<6>(L, valid);
      const uint32_t rk = lanes_below(mm);
      const uint32_t old = valid ? S.run[wave][L] : 0u;
      if (valid && rk == 0) S.run[wave][L] = old + (uint32_t)__popcll(mm);
      pk[it] = L | ((old + rk) << 6);
    }
    __syncthreads();
    if (wave == 0) {
      // per length: prefix over waves, then the block's length-sorted starts
      uint32_t tot = 0;
      if (lane < (uint32_t)kNB) {
        for (int v = 0; v < NW; ++v) {
          const uint32_t t = S.run[v][lane];
          S.run[v][lane] = tot;
          tot += t;
        }
      }
      const uint32_t ex = wave_incl_scan(tot) - tot;
      if (lane <= (uint32_t)kNB) S.bstart[lane] = ex;
      if (lane < (uint32_t)kNB) S.dst[lane] -= ex;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const uint32_t i = wofs + it * 64 + lane;
      if (i < nw) {
        const uint32_t L = pk[it] & 63u;
        S.slot[S.bstart[L] + S.run[wave][L] + (pk[it] >> 6)] = (uint16_t)i;
      }
    }
    __syncthreads();
    // class c holds lengths (8(c-1), 8c] (class 0: 0..4); its slots start at
    // the bucket start of its shortest length
    const uint32_t cpos = lead - c0;                 // LDS byte of character position a is a + cpos
    const uint32_t ibase = r.ws - w.doc_off[r.doc];  // document-relative index of the block's first word
    const uint32_t q1 = S.bstart[5], q2 = S.bstart[9], q3 = S.bstart[17], q4 = S.bstart[25];
    scatter_class<NT, 0>(w, S, s_off, 0, q1, staged, cpos, ibase, chars);
    scatter_class<NT, 1>(w, S, s_off, q1, q2, staged, cpos, ibase, chars);
    scatter_class<NT, 2>(w, S, s_off, q2, q3, staged, cpos, ibase, chars);
    scatter_class<NT, 3>(w, S, s_off, q3, q4, staged, cpos, ibase, chars);
    scatter_class<NT, 4>(w, S, s_off, q4, nw, staged, cpos, ibase, chars);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- k_pack_full
// Baseline without length lists: every word of the (single) document becomes
// one 32-byte key, its length in the top byte followed by up to 31 of its
// bytes, written at its input position; the whole list is then sorted as one
// segment.  Comparing such keys (then the index) is the same total order as
// the bucketed sort's, so the result is identical.  A word longer than 31
// bytes does not fit the key and is reported as too long.
template <int NT>
__global__ __launch_bounds__(NT) void k_pack_full(Ws w) {
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t N = h->n_words;
  const uint32_t* off = h->d.offsets;
  const uint8_t* chars = h->d.chars;
  uint32_t bad = 0;
  for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < N; i += gridDim.x * NT) {
    const uint32_t a = off[i], L = off[i + 1] - a;
    if (L > (uint32_t)kMaxLen - 1) {
      bad = 1;
      continue;
    }
    uint64_t ln[4];
    load_be_lanes<4>(chars + a, L, ln);
    const uint64_t top = (uint64_t)L << 56;
    w.a.k[3][i] = (ln[2] << 56) | (ln[3] >> 8);
    w.a.k[2][i] = (ln[1] << 56) | (ln[2] >> 8);
    w.a.k[1][i] = (ln[0] << 56) | (ln[1] >> 8);
    w.a.k[0][i] = top | (ln[0] >> 8);
    w.a.idx[i] = i;
  }
  if (__any(bad)) {
    if (__lane_id() == 0) {
      atomicOr(&h->status, ST_TOO_LONG);
      atomicOr(&h->abort, 1u);
    }
  }
}

// ---------------------------------------------------------------- chunk sort
// Odd-even transposition (the parallel form of bubble sort's adjacent
// compare-exchanges, section 2) on chunks of C consecutive items of a tile.
// Thread t of the workgroup holds items t*E .. t*E+E-1 in registers; C is a
// power of two in [2, NT*E], so a chunk is either inside one thread (C <= E:
// an odd pair (2k+1, 2k+2) is skipped where 2k+2 starts a chunk), spread over
// C/E lanes of one wave (E < C <= 64E: the neighbours at a thread edge are
// exchanged with wave shuffles), or over C/(64E) waves (C > 64E: the
// neighbours at a wave edge go through LDS, two barriers a phase).  C phases
// sort a chunk; the loop also stops early once an even and an odd phase
// exchange nothing (in the wave, or in the workgroup when chunks span waves),
// bubble sort's own stopping rule.  Every thread of the workgroup must call
// it with the same C.
template <int NT, class K, int E>
__device__ inline void oddeven_chunks(K (&e)[E], uint32_t C) {
  constexpr int NW = NT / 64;
  __shared__ K s_first[NW], s_last[NW];
  __shared__ uint32_t s_any[2];
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const bool cross = C > (uint32_t)E;             // chunks span threads
  const bool waves = C > 64u * E;                 // ... and waves (block-uniform)
  const uint32_t first = threadIdx.x * E;          // tile index of this thread's first item
  const bool has_next = cross && threadIdx.x + 1 < (uint32_t)NT && ((first + E) & (C - 1)) != 0;
  const bool has_prev = cross && threadIdx.x > 0 && (first & (C - 1)) != 0;
  if (waves && threadIdx.x == 0) s_any[0] = 0;
  for (uint32_t p = 0, par = 0; p < C; p += 2, par ^= 1) {
    bool sw = false;
#pragma unroll
    for (int j = 0; j + 1 < E; j += 2) sw |= e_cmp_xchg(e[j], e[j + 1]);
#pragma unroll
    for (int j = 1; j + 1 < E; j += 2)
      if (cross || ((uint32_t)(j + 1) & (C - 1)) != 0) sw |= e_cmp_xchg(e[j], e[j + 1]);
    if (cross) {
      K nx = e_dpp<kDppNext>(e[0]);
      K pv = e_dpp<kDppPrev>(e[E - 1]);
      if (waves) {
        if (lane == 0) s_first[wave] = e[0];
        if (lane == 63) s_last[wave] = e[E - 1];
        __syncthreads();
        // every thread has read the previous iteration's flag before this
        // barrier, so its slot may be cleared for the next iteration
        if (threadIdx.x == 0) s_any[par ^ 1] = 0;
        if (lane == 63 && wave + 1 < (uint32_t)NW) nx = s_first[wave + 1];
        if (lane == 0 && wave > 0) pv = s_last[wave - 1];
      }
      // without `waves`, lane 63 never has its next item in its chunk (64E is
      // a multiple of C), nor lane 0 its previous one
      if (has_next && e_less(nx, e[E - 1])) {
        e[E - 1] = nx;
        sw = true;
      }
      if (has_prev && e_less(e[0], pv)) e[0] = pv;
    }
    if (waves) {
      if (__any(sw) && lane == 0) atomicOr(&s_any[par], 1u);
      __syncthreads();
      if (!s_any[par]) break;   // the same value in every thread
    } else if (!__any(sw)) {
      break;
    }
  }
}

// Accessor of a sorted run held contiguously in LDS.
template <class Tile>
struct LinRun {
  const Tile& t;
  int base;
  __device__ typename Tile::value_type operator()(int i) const { return t.get(base + i); }
};
// Bit length of x (0 for 0): 2^bitlen(x) - 1 >= x.
__device__ inline int bitlen(uint32_t x) { return 32 - (int)__clz(x); }

// Merge path (Odeh et al., "Merge Path - Parallel Merging Made Simple", 2012):
// number of A items among the first d outputs of the stable merge of A and B
// (A first on ties).  Binary search by one thread.
template <class RA, class RB>
__device__ inline int run_merge_path(const RA& A, int la, const RB& B, int lb, int d) {
  int lo = d > lb ? d - lb : 0;
  int hi = d < la ? d : la;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (!e_less(B(d - 1 - mid), A(mid)))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// The same search by K halving steps, where 2^K - 1 >= min(la, lb) bounds the
// search range.  With K the same for the whole wave the loop does not
// diverge; each step reads A and B at indices clamped into the runs and only
// counts when the probe lies in range, so no step branches on data.  A[0] and
// B[0] must be readable.
template <class RA, class RB>
__device__ inline int run_merge_path_steps(const RA& A, int la, const RB& B, int lb, int d, int K) {
  int lo = d > lb ? d - lb : 0;
  const int hi = d < la ? d : la;
  for (int k = K - 1; k >= 0; --k) {
    const int a = lo + (1 << k) - 1;   // lo advances by 2^k when A[a] precedes B[d-1-a]
    const int ai = a < la ? a : (la > 0 ? la - 1 : 0);
    const int bi = d - 1 - a > 0 ? d - 1 - a : 0;
    const bool take = a < hi && !e_less(B(bi), A(ai));
    lo = take ? lo + (1 << k) : lo;
  }
  return lo;
}

// The E smallest items of A[ai..ai+E) and B[bi..bi+E), in order, into
// registers: the candidates are loaded independently (no dependent load
// chain), min(x[i], y[E-1-i]) keeps the E smallest as a bitonic sequence
// (half-cleaner of x followed by y reversed), and log2(E) half-cleaner stages
// sort it (Batcher's bitonic merge).  Items past a run's end read as the
// sentinel.
template <class K, int E, class RA, class RB>
__device__ inline void run_bitonic_merge(const RA& A, int la, const RB& B, int lb, int ai, int bi, K (&out)[E]) {
  K x[E], y[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    x[i] = ai + i < la ? A(ai + i) : e_sentinel<K>();
    y[i] = bi + i < lb ? B(bi + i) : e_sentinel<K>();
  }
#pragma unroll
  for (int i = 0; i < E; ++i) out[i] = e_select(e_less(y[E - 1 - i], x[i]), y[E - 1 - i], x[i]);
#pragma unroll
  for (int st = E / 2; st >= 1; st >>= 1) {
#pragma unroll
    for (int i = 0; i < E; ++i)
      if ((i & st) == 0) e_cmp_xchg(out[i], out[i + st]);
  }
}

// Merge path over two runs held contiguously in LDS.
template <class Tile>
__device__ inline int lds_merge_path(const Tile& t, int a0, int la, int b0, int lb, int d) {
  return run_merge_path(LinRun<Tile>{t, a0}, la, LinRun<Tile>{t, b0}, lb, d);
}

// The diagonal search and the E outputs on a merge tile laid out with
// sentinels: run A at [0, la), a sentinel at la, run B at [la+1, la+1+lb), a
// sentinel after it, and at least E more readable slots.  Reads past both sentinels only feed
// outputs beyond the tile's count, which are never stored, so the serial
// merge needs no clamping.
template <class Tile>
__device__ inline int padded_merge_path(const Tile& t, int la, int lb, int d) {
  return run_merge_path_steps(LinRun<Tile>{t, 0}, la, LinRun<Tile>{t, la + 1}, lb, d,
                              bitlen((uint32_t)(la < lb ? la : lb)));
}

template <int E, class Tile>
__device__ inline void padded_serial_merge(const Tile& t, int la, int ai, int bi,
                                           typename Tile::value_type (&out)[E]) {
  using K = typename Tile::value_type;
  int pa = ai, pb = la + 1 + bi;
  K ha = t.get(pa), hb = t.get(pb);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const bool takeB = e_less(hb, ha);
    out[j] = e_select(takeB, hb, ha);
    pa += takeB ? 0 : 1;
    pb += takeB ? 1 : 0;
    const K nv = t.get(takeB ? pb : pa);
    ha = e_select(takeB, ha, nv);
    hb = e_select(takeB, nv, hb);
  }
}

template <int E, int MM, class Tile>
__device__ inline void padded_register_merge(const Tile& t, int la, int lb, int ai, int bi,
                                             typename Tile::value_type (&out)[E]) {
  if (MM == 0)
    padded_serial_merge<E>(t, la, ai, bi, out);
  else
    run_bitonic_merge(LinRun<Tile>{t, 0}, la, LinRun<Tile>{t, la + 1}, lb, ai, bi, out);
}

// One merge round in registers for runs of M*E items held by M neighbouring
// lanes each (blocked: lane l holds items l*E .. l*E+E-1 of the pair), the
// pair of runs in 2M aligned lanes: Batcher's bitonic merge.  Item i of the
// first run meets item 2ME-1-i of the second (the mirror lane, the item
// reversed), the lower half keeping the smaller; then half-cleaners at lane
// distance M/2 .. 1 (same item index, the lower lane keeping the smaller)
// and at item distance E/2 .. 1 inside each lane.  Afterwards the 2M lanes
// hold the merged run in blocked order.  M is 1 or 2 (quad permutes); every
// lane of the wave takes part.
template <int M, class K, int E>
__device__ inline void lane_merge_round(K (&e)[E]) {
  static_assert(M == 1 || M == 2, "pairs of runs inside a quad");
  constexpr int kMirror = M == 1 ? 0xB1 : 0x1B;   // quad_perm: lane ^ 1, lane ^ 3
  constexpr int kSwap1 = 0xB1;
  const uint32_t lane = __lane_id();
  {
    // items r and E-1-r together: both partner values are read before
    // either is replaced (the partner lane runs the same instructions)
    const bool upper = (lane & M) != 0;
#pragma unroll
    for (int r = 0; r < E / 2; ++r) {
      const K a = e_dpp<kMirror>(e[E - 1 - r]);
      const K b = e_dpp<kMirror>(e[r]);
      e[r] = e_select(e_less(a, e[r]) != upper, a, e[r]);
      e[E - 1 - r] = e_select(e_less(b, e[E - 1 - r]) != upper, b, e[E - 1 - r]);
    }
  }
  if (M == 2) {
    const bool upper = (lane & 1) != 0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const K q = e_dpp<kSwap1>(e[r]);
      e[r] = e_select(e_less(q, e[r]) != upper, q, e[r]);
    }
  }
#pragma unroll
  for (int st = E / 2; st >= 1; st >>= 1) {
#pragma unroll
    for (int i = 0; i < E; ++i)
      if ((i & st) == 0) e_cmp_xchg(e[i], e[i + st]);
  }
}

// Sorting core of a tile held as E items per thread in registers (blocked:
// thread t holds items t*E..t*E+E-1 of the tile): odd-even transposition on
// chunks of C, then (unless only the chunks are wanted) the merge of the
// sorted chunks -- inside a thread's registers while runs are shorter than E,
// then merge-path rounds through LDS until one run covers the tile's cnt real
// items (the rest of the tile is the fill, key_fill, already in place: above
// every real key, below the sentinel).
// In the round that merges runs of R, item i sits in slot i + i/R: every run
// is followed by a sentinel slot, so the serial merge reads one slot per
// output without a bounds test (its positions only reach a run's sentinel
// once the run is used up).  The tile must hold T + T/E slots.
template <int NT, int E, int MM, class Tile>
__device__ inline void sort_tile_core(Tile& tile, typename Tile::value_type (&e)[E], uint32_t C, uint32_t cnt,
                                      bool merge = true) {
  using K = typename Tile::value_type;
  constexpr int T = NT * E;
  oddeven_chunks<NT>(e, C);
  if (!merge) return;
  // runs of C inside a thread are merged there by the same transposition on
  // all E items (the merge strategy is free: the result is unique)
  if (C < (uint32_t)E) oddeven_chunks<NT>(e, (uint32_t)E);
  uint32_t R0 = C < (uint32_t)E ? (uint32_t)E : C;
  // the rounds whose pairs of runs lie in two neighbouring lanes (up to 16
  // items a thread) and in four (up to 8) in registers: no LDS round trip,
  // no barrier; with 16 items the four-lane round costs about what an LDS
  // round does
  if (E <= 16 && R0 == (uint32_t)E && R0 < (uint32_t)T && R0 < cnt) {
    lane_merge_round<1>(e);
    R0 <<= 1;
  }
  if (E <= 8 && R0 == 2u * E && R0 < (uint32_t)T && R0 < cnt) {
    lane_merge_round<2>(e);
    R0 <<= 1;
  }
  for (uint32_t R = R0; R < (uint32_t)T && R < cnt; R <<= 1) {
    const int lr = __ffs((int)R) - 1;   // R is a power of two, at least E
    const int o = threadIdx.x * E;
    const int g = o + (o >> lr);        // a thread's E items lie inside one run
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) tile.put(g + r, e[r]);
    if (((o + E) & (int)(R - 1)) == 0) tile.put(g + E, e_sentinel<K>());
    __syncthreads();
    const int p0 = o & ~(int)(2 * R - 1);
    const int d = o - p0;
    const int sa = p0 + (p0 >> lr), sb = sa + (int)R + 1;
    const int a = lds_merge_path(tile, sa, (int)R, sb, (int)R, d);
    if (MM == 0) {
      // Every item of a run (the fill included) lies strictly below the
      // sentinel slot that ends it, so a run at its sentinel is taken only
      // when the other is at its own, i.e. after all 2R outputs: a position
      // advances only from a run's item and never passes the sentinel slot.
      int pa = sa + a, pb = sb + (d - a);
      K ha = tile.get(pa), hb = tile.get(pb);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const bool takeB = e_less(hb, ha);
        e[j] = e_select(takeB, hb, ha);
        const int nxt = (takeB ? pb : pa) + 1;   // the taken run's next slot
        pa = takeB ? pa : nxt;
        pb = takeB ? nxt : pb;
        const K nv = tile.get(nxt);
        ha = e_select(takeB, ha, nv);
        hb = e_select(takeB, nv, hb);
      }
    } else {
      run_bitonic_merge(LinRun<Tile>{tile, sa}, (int)R, LinRun<Tile>{tile, sb}, (int)R, a, d - a, e);
    }
  }
}

// Merge path on a diagonal over global memory, by groups of K lanes (K
// divides 64): each group finds the split of its own diagonal, K probes per
// round.  Fewer probes per round
// touch fewer cache lines; more rounds cost latency.
template <int NL, int K>
__device__ inline uint32_t group_merge_path(const KeyBuf& buf, size_t a_base, uint32_t la, size_t b_base,
                                            uint32_t lb, uint32_t d, bool active) {
  const uint32_t lane = __lane_id();
  const uint32_t gl = lane % K;
  const uint64_t gmask = K == 64 ? ~0ull : (((1ull << K) - 1) << (lane - gl));
  uint32_t lo = 0, hi = 0;
  if (active) {
    lo = d > lb ? d - lb : 0u;
    hi = d < la ? d : la;
  }
  while (__any(lo < hi)) {
    const uint32_t step = (hi - lo + K - 1) / K;
    const uint32_t a = lo + gl * step;
    bool p = false;
    if (lo < hi && a < hi) {
      const Key<NL> A = gload<NL>(buf, a_base + a);
      const Key<NL> B = gload<NL>(buf, b_base + (d - 1 - a));
      p = !key_less<NL>(B, A);
    }
    const uint32_t c = __popcll(__ballot(p) & gmask);
    if (lo < hi) {
      if (c == 0) {
        hi = lo;
      } else {
        const uint32_t nlo = lo + (c - 1) * step + 1;
        hi = min(lo + c * step, hi);
        lo = nlo;
      }
    }
  }
  return lo;
}

// Segment of a tile from the device lists: k-th segment of the class sublist
// whose tile prefix covers t.
struct TileSeg {
  uint32_t base, n, j;
};
__device__ inline TileSeg find_tile(const Ws& w, const uint32_t* prefix, uint32_t cstart, uint32_t count,
                                    uint32_t t) {
  const uint32_t k = wave_find(prefix, count, t);
  const uint32_t s = w.sorted[cstart + k];
  TileSeg r;
  r.base = w.seg_base[s];
  r.n = w.seg_n[s];
  r.j = t - prefix[k];
  return r;
}

// ---------------------------------------------------------------- k_sort_tiles
// Chunk sort of one tile of T = NT*E items of a segment (class cls), then
// merges in LDS up to T.  A segment that fits one tile is finished here and
// its indices go straight to the output permutation; otherwise the sorted
// tile is written back in place for the merge levels.
template <int NL, int NT, int E, int MM>
__global__ __launch_bounds__(NT) void k_sort_tiles(Ws w, int cls, TileWork tw) {
  constexpr int T = NT * E;
  __shared__ LdsTile<NL, T + T / E> tile;
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t C = w.chunk[cls];   // a power of two in [2, 1024], at most T
  uint32_t ntiles, cstart = 0, ccount = 0;
  const uint32_t* st = nullptr;
  if (tw.direct) {
    ntiles = (tw.n + T - 1) / T;
  } else {
    cstart = h->cls_start[cls];
    ccount = h->pack_start[cls] - cstart;
    st = w.st + cstart + cls;
    ntiles = h->sort_tiles[cls];
  }
  uint32_t* out_perm = h->d.out_perm;
  const bool keep = h->d.out_text != nullptr;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    TileSeg g;
    if (tw.direct) {
      g.base = tw.base;
      g.n = tw.n;
      g.j = t;
    } else {
      g = find_tile(w, st, cstart, ccount, t);
    }
    const uint32_t lo = g.j * T;
    const uint32_t cnt = min((uint32_t)T, g.n - lo);
    // only the chunks: every tile writes its chunk-sorted indices (the
    // segment's runs of C are not merged)
    const bool final = g.n <= (uint32_t)T || tw.chunks_only;
    const size_t gb = (size_t)g.base + lo;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const uint32_t i = threadIdx.x + r * NT;
      tile.put(i, i < cnt ? gload<NL>(w.a, gb + i) : key_fill<NL>());
    }
    __syncthreads();
    Key<NL> e[E];
#pragma unroll
    for (int r = 0; r < E; ++r) e[r] = tile.get(threadIdx.x * E + r);
    sort_tile_core<NT, E, MM>(tile, e, C, cnt, !tw.chunks_only);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) tile.put(threadIdx.x * E + r, e[r]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const uint32_t i = threadIdx.x + r * NT;
      if (i < cnt) {
        const Key<NL> v = tile.get(i);
        if (final) out_perm[gb + i] = key_index<NL>(v);
        if ((!final || keep) && !tw.chunks_only) gstore<NL>(w.a, gb + i, v);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- k_sort_packed
// Short segments (at most kPackMax = kPackTile/2 words, all finished by the
// chunk sort) are sorted several to a tile.  The class's short segments are
// laid end to end in a virtual sequence (their sizes' prefix); packed tile k
// takes every segment that starts in [k*kPackMax, (k+1)*kPackMax), at most
// kPackTile items.  Each item carries its segment's ordinal in the tile as a
// tag compared before the key, so sorting the tile (odd-even chunks, then
// merge path in LDS) sorts every segment in place; item p of the sorted tile
// belongs to the segment its tag names.
template <int NL, int E, int MM>
__global__ __launch_bounds__(kPackTile / E) void k_sort_packed(Ws w, int cls) {
  constexpr int NT = kPackTile / E;
  constexpr uint32_t H = kPackMax;
  __shared__ TLdsTile<NL, kPackTile + kPackTile / E> tile;
  __shared__ uint32_t s_start[kPackMax + 1];   // segment starts inside the tile
  __shared__ uint32_t s_base[kPackMax];        // segment first output positions
  __shared__ uint32_t s_rng[3];
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t C = w.chunk[cls];   // a power of two in [2, 1024], at most kPackTile
  const uint32_t ps = h->pack_start[cls];
  const uint32_t npack = h->cls_start[cls + 1] - ps;
  const uint32_t* vp = w.vpre + ps + cls;     // npack + 1 entries
  const uint32_t ntiles = (h->pack_words[cls] + H - 1) / H;
  uint32_t* out_perm = h->d.out_perm;
  const bool keep = h->d.out_text != nullptr;
  for (uint32_t k = blockIdx.x; k < ntiles; k += gridDim.x) {
    if (threadIdx.x < 2) {
      // first segment starting at or after k*H (resp. (k+1)*H)
      const uint32_t x = (k + threadIdx.x) * H;
      uint32_t lo = 0, hi = npack;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (vp[mid] < x)
          lo = mid + 1;
        else
          hi = mid;
      }
      s_rng[threadIdx.x] = lo;
    }
    __syncthreads();
    const uint32_t first = s_rng[0], last = s_rng[1];
    const uint32_t nseg = last - first;
    const uint32_t v0 = vp[first];
    const uint32_t cnt = vp[last] - v0;
    for (uint32_t j = threadIdx.x; j < nseg; j += NT) {
      s_start[j] = vp[first + j] - v0;
      s_base[j] = w.seg_base[w.sorted[ps + first + j]];
    }
    if (threadIdx.x == 0) s_start[nseg] = cnt;
    __syncthreads();
    TKey<NL> e[E];
    if (nseg) {
      // segment of this thread's first item, then walk forward
      const uint32_t p0 = threadIdx.x * E;
      uint32_t lo = 0, hi = nseg;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_start[mid] <= p0)
          lo = mid;
        else
          hi = mid;
      }
      uint32_t tg = lo;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const uint32_t p = p0 + r;
        if (p < cnt) {
          while (s_start[tg + 1] <= p) ++tg;
          e[r].k = gload<NL>(w.a, (size_t)s_base[tg] + (p - s_start[tg]));
          e[r].tag = tg;
        } else {
          e_set_fill(e[r]);
        }
      }
      sort_tile_core<NT, E, MM>(tile, e, C, cnt);
      if (keep) __syncthreads();   // every item read before any is overwritten
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const uint32_t p = p0 + r;
        if (p < cnt) {
          const size_t q = (size_t)s_base[e[r].tag] + (p - s_start[e[r].tag]);
          out_perm[q] = key_index<NL>(e[r].k);
          if (keep) gstore<NL>(w.a, q, e[r].k);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- merge levels
// The tiles' geometry (merge_tile, TileRec, tile_io, the placement
// bookkeeping) is in sw_tiles.hpp.

// Merge tiles are placed by groups of kPartLanes lanes (kPartLanes probes per
// round of the merge-path search): fewer lanes touch fewer cache lines in
// all (a probe is a cache line until the last rounds), more lanes need fewer
// rounds.  The rounds' latency hides behind the other classes' kernels, so
// 8 lanes beat 16 (and 16 beat 32 and 64); 4 lanes ran the c4 pass in the
// same time.
constexpr int kPartLanes = 8;

// A tile's inputs are read once per level: nontemporal loads (measured 2 %
// faster on the c4 merge levels than plain loads).
template <int NL, int NT, int E>
__device__ inline void load_tile_regs(const KeyBuf& src, const TileIO& io, Key<NL> (&pf)[E]) {
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = threadIdx.x + r * NT;
    if (i < io.na)
      pf[r] = gload_nt<NL>(src, io.apos + i);
    else if (i < io.cnt)
      pf[r] = gload_nt<NL>(src, io.bpos + (i - io.na));
  }
}

// ---------------------------------------------------------------- k_merge
// One merge level of class cls: every segment still merging has runs of
// R = T << level sorted items; pairs of runs are merged into runs of 2R.
// Work is cut into tiles of P = NT*E outputs; a workgroup takes a contiguous
// range of tiles and places them itself, TB at a time: group g of
// kPartLanes lanes finds the segment of tile t0+g (a kPartLanes-ary search
// over the class's tile prefix) and the merge-path split at its first output,
// so that the split at a tile's last output is the next tile's (NT/kPartLanes
// searches place NT/kPartLanes - 1 tiles; groups past the split after the
// range's last tile search nothing).  Tiles then run as a pipeline:
// while tile k merges, the inputs of tile k+1 are already on their way into
// registers.  A tile's two input ranges are staged in LDS as A, sentinel, B,
// sentinel; each thread finds its diagonal by merge path and merges E
// outputs in registers (method MM); the outputs are staged back in LDS and
// stored in order with the nontemporal hint.  The segment's last level writes
// indices to the output permutation.
template <int NL, int NT>
__device__ inline void place_tiles(const Ws& w, int cls, int level, const TileWork& tw, uint32_t P, uint32_t ntiles,
                                   uint32_t t0, uint32_t t_end, TileRec* s_rec, uint32_t* s_split) {
  constexpr int NG = NT / kPartLanes;
  static_assert(NG >= 2 && NG <= 64, "groups of kPartLanes lanes");
  Header* h = w.h;
  const uint64_t R = (uint64_t)w.T[cls] << level;
  const uint32_t lane = __lane_id();
  const uint32_t g = threadIdx.x / kPartLanes;
  const uint32_t t = t0 + g;
  const bool active = place_group_active(t0, g, ntiles, t_end);
  TileSeg sg{0, 0, 0};
  if (tw.direct) {
    sg.base = tw.base;
    sg.n = tw.n;
    sg.j = t;
  } else {
    // the tile's segment: the last k with mt[k] <= t, kPartLanes probes per
    // round (every lane of the group takes part, active or not)
    const uint32_t cstart = h->cls_start[cls];
    const uint32_t cact = h->active[cls][level];
    const uint32_t* mt = w.mt + cstart + cls;
    const uint32_t gl = lane % kPartLanes;
    const uint64_t gmask = (((1ull << kPartLanes) - 1) << (lane - gl));
    KarySearch ks{0, active ? cact : 1u};
    while (__any(ks.open())) {
      const uint32_t k = ks.probe(gl, kPartLanes);
      const bool p = ks.open() && k < ks.hi && mt[k] <= t;
      const uint32_t c = __popcll(__ballot(p) & gmask);
      if (ks.open()) ks.narrow(c, kPartLanes);   // mt[lo] <= t, so c >= 1
    }
    if (active) {
      const uint32_t s = w.sorted[cstart + ks.lo];
      sg.base = w.seg_base[s];
      sg.n = w.seg_n[s];
      sg.j = t - mt[ks.lo];
    }
  }
  MergeTile m{};
  if (active) m = merge_tile(sg.n, sg.j, R, P);
  const KeyBuf src = (level & 1) ? w.b : w.a;
  const size_t abase = (size_t)sg.base + m.ps;
  const uint32_t sp = group_merge_path<NL, kPartLanes>(src, abase, m.la, abase + m.la, m.lb, m.d0, active);
  if (active && lane % kPartLanes == 0) {
    s_split[g] = sp;
    if (g + 1 < (uint32_t)NG) s_rec[g] = TileRec{sg.base, sg.n, sg.j, sp};
  }
}

template <int NL, int NT, int E, int MM>
__global__ __launch_bounds__(NT) void k_merge(Ws w, int cls, int level, TileWork tw) {
  constexpr int P = NT * E;
  constexpr uint32_t TB = NT / kPartLanes - 1;   // tiles placed per batch
  __shared__ LdsTile<NL, P + 2 * E> tile;
  __shared__ TileRec s_rec[TB];
  __shared__ uint32_t s_split[TB + 1];
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t Tc = w.T[cls];
  const uint64_t R = (uint64_t)Tc << level;
  uint32_t ntiles;
  if (tw.direct) {
    if ((uint32_t)level >= tw.m) return;
    ntiles = (tw.n + P - 1) / P;
  } else {
    const uint32_t cact = h->active[cls][level];
    ntiles = cact ? (w.mt + h->cls_start[cls] + cls)[cact] : 0u;
  }
  // this workgroup's tiles: [tb, tb + nb), the ranges balanced over the grid
  const uint32_t G = gridDim.x, q = ntiles / G, rem = ntiles % G;
  const uint32_t nb = q + (blockIdx.x < rem ? 1u : 0u);
  if (nb == 0) return;
  const uint32_t tb = blockIdx.x * q + min(blockIdx.x, rem);
  const KeyBuf src = (level & 1) ? w.b : w.a;
  const KeyBuf dst = (level & 1) ? w.a : w.b;
  uint32_t* out_perm = h->d.out_perm;
  const bool keep = h->d.out_text != nullptr;

  place_tiles<NL, NT>(w, cls, level, tw, P, ntiles, tb, tb + nb, s_rec, s_split);
  __syncthreads();
  TileIO cur = tile_io(s_rec[0], s_split[1], R, P, Tc, level);
  Key<NL> pf[E];
  load_tile_regs<NL, NT, E>(src, cur, pf);
  for (uint32_t k = 0; k < nb; ++k) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = threadIdx.x + r * NT;
      if (i < cur.cnt) tile.put(i < cur.na ? i : i + 1, pf[r]);
    }
    if (threadIdx.x == 0) {
      tile.put(cur.na, key_sentinel<NL>());
      tile.put(cur.cnt + 1, key_sentinel<NL>());
    }
    const bool has_next = k + 1 < nb;
    const uint32_t kn = place_slot(k + 1, TB);   // the next tile's slot in its batch
    if (has_next && kn == 0) place_tiles<NL, NT>(w, cls, level, tw, P, ntiles, tb + k + 1, tb + nb, s_rec, s_split);
    __syncthreads();
    TileIO nxt = cur;
    if (has_next) {
      nxt = tile_io(s_rec[kn], s_split[kn + 1], R, P, Tc, level);
      load_tile_regs<NL, NT, E>(src, nxt, pf);
    }
    const int cnt = cur.cnt, na = cur.na, nbv = cnt - na;
    const int diag = threadIdx.x * E;
    Key<NL> e[E];
    if (diag < cnt) {
      const int sa = padded_merge_path(tile, na, nbv, diag);
      padded_register_merge<E, MM>(tile, na, nbv, sa, diag - sa, e);
    }
    __syncthreads();
    if (diag < cnt) {
#pragma unroll
      for (int r = 0; r < E; ++r) tile.put(diag + r, e[r]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int o = threadIdx.x + r * NT;
      if (o < cnt) {
        const Key<NL> v = tile.get(o);
        if (cur.final) __builtin_nontemporal_store(key_index<NL>(v), out_perm + cur.ob + o);
        if (!cur.final || keep) gstore_nt<NL>(dst, cur.ob + o, v);
      }
    }
    __syncthreads();
    cur = nxt;
  }
}

// ---------------------------------------------------------------- four-way split
// Co-ranks sp[] of rank d in the four runs (start st[r], len[r]) by the
// bracket search of sw_split.hpp: each round every slot of every run is
// sampled by one thread, every interior sample judged by one thread, and the
// brackets narrowed with LDS atomics.  False if the search did not close
// (never expected; the caller then stops its work and flags the run).
template <int NL>
struct KeyLess {
  __host__ __device__ __attribute__((always_inline)) bool operator()(const Key<NL>& a, const Key<NL>& b) const {
    return key_less<NL>(a, b);
  }
};
template <int NL, int NT>
__device__ __attribute__((always_inline)) inline bool split4(SplitScratch<Key<NL>>& S, const KeyBuf& src,
                                                             const uint64_t (&st)[4], const uint32_t (&len)[4],
                                                             uint32_t d, uint32_t (&sp)[4]) {
  if (threadIdx.x == 0) {
    split_init(S, len, d);
#pragma unroll
    for (int i = 0; i < 4; ++i) S.start[i] = st[i];
  }
  __syncthreads();
  while (!S.done) {
    if (S.rounds >= (uint32_t)kSplitMaxRounds) return false;   // the same in every thread
    for (uint32_t slot = threadIdx.x; slot < (uint32_t)(kSplitRuns * kSplitSlots); slot += NT) {
      const int i = (int)(slot / kSplitSlots), j = (int)(slot % kSplitSlots);
      const uint32_t p = split_slot_pos(S, i, j);
      S.pos[i][j] = p;
      if (p != kSplitNone) S.key[i][j] = gload<NL>(src, (size_t)(S.start[i] + p));
    }
    if (threadIdx.x == 0) split_begin_round(S);
    __syncthreads();
    for (uint32_t slot = threadIdx.x; slot < (uint32_t)(kSplitRuns * kSplitSlots); slot += NT) {
      const int i = (int)(slot / kSplitSlots), j = (int)(slot % kSplitSlots);
      if (j == 0 || j == kSplitSlots - 1 || S.pos[i][j] == kSplitNone) continue;
      const int v = split_decide(S, i, j, KeyLess<NL>());
      if (v < 0) atomicMax(&S.newlo[i], S.pos[i][j] + 1);
      if (v > 0) atomicMin(&S.newhi[i], S.pos[i][j]);
    }
    __syncthreads();
    if (threadIdx.x == 0) split_finish_round(S);
    __syncthreads();
  }
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sp[i] = S.lo[i];
    sum += sp[i];
  }
  __syncthreads();   // the scratch may share LDS with the caller's buffers
  return sum == d;
}

// ---------------------------------------------------------------- k_merge4w
// One four-way merge pass of class cls by bounded windows (sw_window.hpp):
// groups of four runs of R = T * 4^level items merged into runs of 4R.  The
// pass's output (the active segments of the class one after another, or the
// one segment given directly) is cut into one contiguous range per
// workgroup; a range entered inside a group starts from the co-ranks of the
// split search.  A step of W = NT*E/4 items a window:
//   A  the windows loaded during the last step go into LDS (run r from
//      slot r*W);
//   B  waves 0-3 find the bound and count their run's items below it (two
//      rounds of 64 probes);
//   C  the next step's windows are requested into registers;
//   D  threads [0, NT/2) merge X = A and B, the others Y = C and D, E items
//      each from a merge-path diagonal (reads bounded by the counts), into
//      LDS, each followed by a sentinel;
//   E  every thread merges E outputs of X and Y from its diagonal into LDS,
//      and the step's outputs are stored in order (indices to the output
//      permutation on a segment's last pass).
// Four barriers a step; LDS holds the windows, X and Y, and the outputs:
// 12W items.
template <int NL, int NT, int E>
struct W4 {
  static_assert(NT >= 256 && NT % 64 == 0, "waves 0-3 search the four windows");
  static constexpr int W = NT * E / 4;
  static_assert(W % 64 == 0, "a wave's window load stays inside one run");
  static_assert(W <= (int)(kWinLanes * kWinLanes), "two rounds of 64 probes cover a window");
  static constexpr int WS = W;           // window slots of a run
  static constexpr int XS = 2 * W + 1;   // X, Y: up to 2W items and a sentinel
  static constexpr int XOFF = kWinRuns * WS, YOFF = XOFF + XS;
  // E slots a serial merge may step past both sentinels (outputs never
  // stored), then the outputs staged for in-order stores
  static constexpr int SOFF = YOFF + XS + E;
  static constexpr int CAP = SOFF + 4 * W;
  struct Lds {
    LdsTile<NL, CAP> t;
    SplitScratch<Key<NL>> sp;
    uint32_t c[kWinRuns];
    uint32_t seg;
  };
};

// E items merged from positions pa and pb of two runs in LDS that each end
// with a sentinel (ties go to the first run; keys are distinct anyway).
template <int E, class Tile>
__device__ __attribute__((always_inline)) inline void lds_serial_merge(const Tile& t, int pa, int pb,
                                                                       typename Tile::value_type (&out)[E]) {
  using K = typename Tile::value_type;
  K ha = t.get(pa), hb = t.get(pb);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const bool takeB = e_less(hb, ha);
    out[j] = e_select(takeB, hb, ha);
    pa += takeB ? 0 : 1;
    pb += takeB ? 1 : 0;
    const K nv = t.get(takeB ? pb : pa);
    ha = e_select(takeB, ha, nv);
    hb = e_select(takeB, nv, hb);
  }
}

// The same from positions pa < ea and pb < eb (either may start at its end):
// a run read to its end reads as the sentinel.
template <int E, class Tile>
__device__ __attribute__((always_inline)) inline void lds_bounded_merge(const Tile& t, int pa, int ea, int pb, int eb,
                                                                        typename Tile::value_type (&out)[E]) {
  using K = typename Tile::value_type;
  K ha, hb;
  e_set_sentinel(ha);
  e_set_sentinel(hb);
  if (pa < ea) ha = t.get(pa);
  if (pb < eb) hb = t.get(pb);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const bool takeB = e_less(hb, ha);
    out[j] = e_select(takeB, hb, ha);
    pa += takeB ? 0 : 1;
    pb += takeB ? 1 : 0;
    const int np = takeB ? pb : pa;
    K nv;
    e_set_sentinel(nv);
    if (np < (takeB ? eb : ea)) nv = t.get(np);
    ha = e_select(takeB, ha, nv);
    hb = e_select(takeB, nv, hb);
  }
}

// Element r of four wave-uniform values without indexing by a runtime r
// (which would put the array in scratch memory).
template <class T>
__device__ __attribute__((always_inline)) inline T pick4(const T (&a)[4], int r) {
  return r == 0 ? a[0] : (r == 1 ? a[1] : (r == 2 ? a[2] : a[3]));
}

// Run of thread t's u-th window item, (t + u*NT) / W: a constant of the
// unrolled loop when W is a multiple of NT, else the same across a wave.
template <int NT, int W>
__device__ __attribute__((always_inline)) inline int w4_run(int u) {
  return W % NT == 0 ? (u * NT) / W : win_load_run(u, (int)threadIdx.x, NT, W);
}

// The next windows into registers: thread t's u-th item is item
// (t + u*NT) % W of run (t + u*NT) / W's window.
template <int NL, int NT, int E, int W>
__device__ __attribute__((always_inline)) inline void w4_load(const KeyBuf& src, const uint64_t (&st)[4],
                                                              const uint32_t (&len)[4], const uint32_t (&cons)[4],
                                                              Key<NL> (&pf)[E]) {
#pragma unroll
  for (int u = 0; u < E; ++u) {
    const int r = w4_run<NT, W>(u);
    const uint32_t i = pick4(cons, r) + (uint32_t)win_load_pos(u, (int)threadIdx.x, NT, W);
    if (i < pick4(len, r)) pf[u] = gload_nt<NL>(src, (size_t)(pick4(st, r) + i));
  }
}

template <int NL, int NT, int E>
__global__ __launch_bounds__(NT) void k_merge4w(Ws w, int cls, int level, TileWork tw) {
  using G = W4<NL, NT, E>;
  using K = Key<NL>;
  constexpr int W = G::W, WS = G::WS;
  __shared__ typename G::Lds L;
  Header* h = w.h;
  if (h->abort) return;
  const uint32_t Tc = w.T[cls];
  const uint64_t R = (uint64_t)Tc << (2 * level);
  uint64_t total;
  const uint32_t* wp = nullptr;
  uint32_t cstart = 0, cact = 0;
  if (tw.direct) {
    if ((uint32_t)level >= tw.m) return;
    total = tw.n;
  } else {
    cstart = h->cls_start[cls];
    cact = 2 * level < kMaxLev ? h->active[cls][2 * level] : 0u;
    wp = w.wpre + cstart + cls;
    total = cact ? wp[cact] : 0u;
  }
  const uint64_t r0 = total * blockIdx.x / gridDim.x, r1 = total * (blockIdx.x + 1) / gridDim.x;
  if (r0 >= r1) return;
  const KeyBuf src = (level & 1) ? w.b : w.a;
  const KeyBuf dst = (level & 1) ? w.a : w.b;
  uint32_t* out_perm = h->d.out_perm;
  const bool keep = h->d.out_text != nullptr;
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  uint32_t k = 0;
  if (!tw.direct) {
    if (tid < 64) {
      const uint32_t kk = wave_find(wp, cact, (uint32_t)r0);
      if (tid == 0) L.seg = kk;
    }
    __syncthreads();
    k = __builtin_amdgcn_readfirstlane(L.seg);
  }
  for (uint64_t pos = r0; pos < r1;) {
    uint32_t base, n;
    uint64_t segw = 0;
    if (tw.direct) {
      base = tw.base;
      n = tw.n;
    } else {
      while (wp[k + 1] <= pos) ++k;
      const uint32_t sg = w.sorted[cstart + k];
      base = w.seg_base[sg];
      n = w.seg_n[sg];
      segw = wp[k];
    }
    const M4Group g = m4_group(n, pos - segw, R);
    const uint64_t gend = segw + g.start + g.size;
    const uint32_t count = (uint32_t)((gend < r1 ? gend : r1) - pos);
    const bool final = merge_passes(n, Tc, 4) == (uint32_t)level + 1;
    const size_t ob = (size_t)base + g.start + g.d;   // first output position of this piece
    uint64_t st[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) st[r] = (uint64_t)base + g.start + g.run_off[r];
    uint32_t cons[4] = {0, 0, 0, 0};
    if (g.d > 0 && !split4<NL, NT>(L.sp, src, st, g.len, g.d, cons)) {
      if (tid == 0) {
        atomicOr(&h->status, ST_INVALID);
        atomicOr(&h->abort, 1u);
      }
      return;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) cons[r] = __builtin_amdgcn_readfirstlane(cons[r]);
    K pf[E];
    w4_load<NL, NT, E, W>(src, st, g.len, cons, pf);
    for (uint32_t done = 0; done < count;) {
      // A: the windows into LDS
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int r = w4_run<NT, W>(u);
        const int i = win_load_pos(u, (int)tid, NT, W);
        if ((uint32_t)i < win_len(pick4(g.len, r), pick4(cons, r), W)) L.t.put(r * WS + i, pf[u]);
      }
      __syncthreads();
      // B: the bound and each run's count (wave r searches run r)
      if (wave < (uint32_t)kWinRuns) {
        const int r = (int)wave;
        K bk = key_sentinel<NL>();
        const int br = win_bound(g.len, cons, (uint32_t)W, [&](int rr) { return L.t.get(rr * WS + W - 1); },
                                 KeyLess<NL>(), bk);
        const uint32_t wl = win_len(pick4(g.len, r), pick4(cons, r), W);
        uint32_t cnt;
        if (br < 0) {
          cnt = wl;
        } else if (br == r) {
          cnt = (uint32_t)W;
        } else {
          const int p1 = win_probe1(wl, lane);
          const bool b1 = p1 >= 0 && e_less(L.t.get(r * WS + p1), bk);
          const uint32_t k1 = (uint32_t)__popcll(__ballot(b1));
          const int p2 = win_probe2(wl, k1, lane);
          const bool b2 = p2 >= 0 && e_less(L.t.get(r * WS + p2), bk);
          cnt = k1 * win_slice(wl) + (uint32_t)__popcll(__ballot(b2));
        }
        // (no sentinel is written into the window here: other waves may still
        // be reading its last item for the bound)
        if (lane == 0) L.c[r] = cnt;
      }
      __syncthreads();
      // the counts are the same in every lane: readfirstlane keeps them (and
      // all the step's bookkeeping that follows) in scalar registers
      uint32_t c[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) c[r] = __builtin_amdgcn_readfirstlane(L.c[r]);
      const uint32_t nx = c[0] + c[1], ny = c[2] + c[3], ns = nx + ny;
      if (ns == 0) {   // never: the bounding window, or what is left, is taken
        if (tid == 0) {
          atomicOr(&h->status, ST_INVALID);
          atomicOr(&h->abort, 1u);
        }
        return;
      }
      // C: the next step's windows, in flight while this one merges
      uint32_t nc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) nc[r] = cons[r] + c[r];
      if (done + ns < count) w4_load<NL, NT, E, W>(src, st, g.len, nc, pf);
      // D: X = merge(A, B) and Y = merge(C, D)
      K e[E];
      {
        const bool side = tid >= (uint32_t)(NT / 2);
        const int diag = (int)(tid - (side ? NT / 2 : 0)) * E;
        const int la = (int)(side ? c[2] : c[0]), lb = (int)(side ? c[3] : c[1]);
        const int a0 = side ? 2 * WS : 0, b0 = a0 + WS;
        const int o0 = side ? G::YOFF : G::XOFF;
        if (diag < la + lb) {
          const int sa = run_merge_path_steps(LinRun<decltype(L.t)>{L.t, a0}, la, LinRun<decltype(L.t)>{L.t, b0}, lb,
                                              diag, bitlen((uint32_t)(la < lb ? la : lb)));
          lds_bounded_merge<E>(L.t, a0 + sa, a0 + la, b0 + (diag - sa), b0 + lb, e);
#pragma unroll
          for (int j = 0; j < E; ++j)
            if (diag + j < la + lb) L.t.put(o0 + diag + j, e[j]);
        }
        if (tid == 0) L.t.put(G::XOFF + (int)nx, key_sentinel<NL>());
        if (tid == (uint32_t)(NT / 2)) L.t.put(G::YOFF + (int)ny, key_sentinel<NL>());
      }
      __syncthreads();
      // E: the outputs, staged in LDS and stored in order
      const uint32_t take = ns < count - done ? ns : count - done;
      {
        const int diag = (int)tid * E;
        if ((uint32_t)diag < take) {
          const int sx = run_merge_path_steps(LinRun<decltype(L.t)>{L.t, G::XOFF}, (int)nx,
                                              LinRun<decltype(L.t)>{L.t, G::YOFF}, (int)ny, diag,
                                              bitlen(nx < ny ? nx : ny));
          lds_serial_merge<E>(L.t, G::XOFF + sx, G::YOFF + (diag - sx), e);
#pragma unroll
          for (int j = 0; j < E; ++j)
            if ((uint32_t)(diag + j) < take) L.t.put(G::SOFF + diag + j, e[j]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const uint32_t q = tid + (uint32_t)r * NT;
        if (q < take) {
          const K v = L.t.get(G::SOFF + (int)q);
          const size_t o = ob + done + q;
          if (final) __builtin_nontemporal_store(key_index<NL>(v), out_perm + o);
          if (!final || keep) gstore_nt<NL>(dst, o, v);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) cons[r] = nc[r];
      done += ns;
    }
    pos += count;
  }
}

}  // namespace sw
