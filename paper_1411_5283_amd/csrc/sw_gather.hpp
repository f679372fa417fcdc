// sw_gather.hpp -- the serving loop's batch packing on the device.
//
// Admitted requests wait in device memory, each in a block of its own: its
// characters (from its first word's first byte) and, after them at the next
// 256-byte boundary, its n+1 offsets exactly as submitted.  A batch is one
// word list of several documents, so its requests' characters must lie back
// to back and their offsets must count from the batch's first character;
// k_gather builds both from the blocks, one workgroup per piece of at most
// kGatherWords words of one request.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

constexpr uint32_t kGatherWords = 8192;

struct GatherPiece {
  const uint8_t* chars;      // the request's characters in its block
  const uint32_t* offsets;   // the request's offsets in its block (n+1 entries)
  uint32_t k0, k1;           // this piece: words k0..k1-1 of the request
  uint32_t n;                // words of the request
  uint32_t wpos;             // the request's first word in the batch
  uint32_t cpos;             // the request's first character in the batch
};

// Offsets entries k0..k1-1 (and entry n, in the request's last piece) as
// offsets[k] - offsets[0] + cpos, and the characters of words k0..k1-1.
// Neighbouring requests both write the entry between them, with the same
// value (a request's end is the next one's cpos).
template <int NT>
__global__ __launch_bounds__(NT) void k_gather(const GatherPiece* pieces, uint8_t* chars_out,
                                                uint32_t* offsets_out) {
  const GatherPiece p = pieces[blockIdx.x];
  const uint32_t o0 = p.offsets[0];
  const uint32_t last = p.k1 == p.n ? p.k1 + 1 : p.k1;
  for (uint32_t k = p.k0 + threadIdx.x; k < last; k += NT) offsets_out[p.wpos + k] = p.offsets[k] - o0 + p.cpos;
  const uint32_t a = p.offsets[p.k0] - o0, b = p.offsets[p.k1] - o0;
  uint8_t* dst = chars_out + p.cpos;
  for (uint32_t j = a + threadIdx.x; j < b; j += NT) dst[j] = p.chars[j];
}

}  // namespace sw
