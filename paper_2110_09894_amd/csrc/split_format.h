// Split BF16 storage of complex64 tensors (internal header).
//
// In split-BF16 plans every operand of a matrix-core product is stored split
// once, by the kernel that produces it, instead of being split again each time
// a tile of it is loaded.  A tensor of E complex elements (all items included)
// occupies the same 8 E bytes as its complex64 form, as four planes of E BF16
// values starting at element offsets 0, ps, 2 ps, 3 ps:
//   plane 0  hi(re) = rne(re)          plane 1  lo(re) = rne(re - hi(re))
//   plane 2  hi(im) = rne(im)          plane 3  lo(im) = rne(im - hi(im))
// with rne = round to nearest even.  Element e of plane q is at q * ps + e, so
// every element offset of the complex64 form (bit strides, item strides,
// gather offsets) addresses the split form unchanged.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kargs.h"

namespace qx {

__device__ __forceinline__ uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Writes element e of a split tensor (base: plane 0, ps: plane stride in elements).
__device__ __forceinline__ void store_split(uint16_t* __restrict__ base, int64_t ps, int64_t e, QxCplx v) {
  const uint16_t rh = bf16_bits(v.x), ih = bf16_bits(v.y);
  base[e] = rh;
  base[e + ps] = bf16_bits(v.x - bf16_value(rh));
  base[e + 2 * ps] = ih;
  base[e + 3 * ps] = bf16_bits(v.y - bf16_value(ih));
}

}  // namespace qx
