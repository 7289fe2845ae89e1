// Split BF16 storage of complex64 tensors (internal header).
//
// In split-BF16 plans every operand of a matrix-core product is stored split
// once, by the kernel that produces it, instead of being split again each time
// a tile of it is loaded.  Each complex element x = re + i im becomes four BF16
// values ("planes"):
//   plane 0  hi(re) = rne(re)          plane 1  lo(re) = rne(re - hi(re))
//   plane 2  hi(im) = rne(im)          plane 3  lo(im) = rne(im - hi(im))
// with rne = round to nearest even.  The tensor keeps its 8 bytes per element
// and its element offsets (bit strides, item strides, gather offsets): every 8
// consecutive elements form a 64-byte chunk holding plane 0 of the 8, then
// plane 1, 2 and 3, so element e of plane q is the BF16 value at
//   (e >> 3) * 32 + q * 8 + (e & 7).
// A matrix-product tile row of 16 consecutive k is then one 128-byte line.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kargs.h"

namespace qx {

// position of the 64-byte chunk holding element e (in BF16 units)
__host__ __device__ __forceinline__ int64_t split_chunk(int64_t e) { return (e >> 3) << 5; }
__host__ __device__ __forceinline__ int64_t split_off(int64_t e, int q) { return split_chunk(e) + (q << 3) + (e & 7); }

__device__ __forceinline__ uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Writes element e of a split tensor whose storage starts at base.
__device__ __forceinline__ void store_split(uint16_t* __restrict__ base, int64_t e, QxCplx v) {
  const uint16_t rh = bf16_bits(v.x), ih = bf16_bits(v.y);
  uint16_t* __restrict__ c = base + split_off(e, 0);
  c[0] = rh;
  c[8] = bf16_bits(v.x - bf16_value(rh));
  c[16] = ih;
  c[24] = bf16_bits(v.y - bf16_value(ih));
}

}  // namespace qx
