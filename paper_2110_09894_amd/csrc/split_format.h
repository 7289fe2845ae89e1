// Split 16-bit storage of complex64 tensors (internal header).
//
// In split-precision plans every operand of a matrix-core product is stored
// split once, by the kernel that produces it, instead of being split again
// each time a tile of it is loaded.  Each complex element x = re + i im
// becomes four 16-bit values ("planes"):
//   plane 0  hi(re) = rne(re)          plane 1  lo(re) = rne(re - hi(re))
//   plane 2  hi(im) = rne(im)          plane 3  lo(im) = rne(im - hi(im))
// with rne = round to nearest even into BF16 (kind 1), or into FP16 (kind 2)
// after multiplying x by the tensor's power-of-two scale (exact), which keeps
// the tensor inside FP16's range.  The tensor keeps its 8 bytes per element
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

typedef __bf16 qx_bf16x2 __attribute__((ext_vector_type(2)));
typedef float qx_f32x2 __attribute__((ext_vector_type(2)));

// hi = [hi(re) | hi(im) << 16], lo = [lo(re) | lo(im) << 16] of one complex value
__device__ __forceinline__ void split_pair(QxCplx v, uint32_t& hi, uint32_t& lo) {
  const qx_f32x2 x = {v.x, v.y};
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, qx_bf16x2));
  const qx_f32x2 h = {__uint_as_float(hi << 16), __uint_as_float(hi & 0xffff0000u)};
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(x - h, qx_bf16x2));
}

typedef _Float16 qx_f16x2 __attribute__((ext_vector_type(2)));

// FP16 planes of one complex value (already scaled): hi = [hi(re) | hi(im) << 16], lo likewise
__device__ __forceinline__ void split_pair_f16(QxCplx v, uint32_t& hi, uint32_t& lo) {
  const qx_f32x2 x = {v.x, v.y};
  const qx_f16x2 h16 = __builtin_convertvector(x, qx_f16x2);
  hi = __builtin_bit_cast(uint32_t, h16);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(x - __builtin_convertvector(h16, qx_f32x2), qx_f16x2));
}

// Planes of one complex value for storage kind 1 (BF16) or 2 (FP16 of v * scale).
__device__ __forceinline__ void split_value(int kind, float scale, QxCplx v, uint32_t& hi, uint32_t& lo) {
  if (kind == 2) split_pair_f16(QxCplx{v.x * scale, v.y * scale}, hi, lo);
  else split_pair(v, hi, lo);
}

// The scale a producer applies to a kind-2 output (1 when there is none).
__device__ __forceinline__ float out_scale(const float* s) { return s ? *s : 1.f; }

// Packs the planes of two consecutive elements (pairs of split_pair) into plane words:
// w[q] = plane q of element 2j in the low half, of element 2j + 1 in the high half.
__device__ __forceinline__ void split_words(uint32_t hi0, uint32_t lo0, uint32_t hi1, uint32_t lo1, uint32_t (&w)[4]) {
  w[0] = __builtin_amdgcn_perm(hi1, hi0, 0x05040100u);
  w[1] = __builtin_amdgcn_perm(lo1, lo0, 0x05040100u);
  w[2] = __builtin_amdgcn_perm(hi1, hi0, 0x07060302u);
  w[3] = __builtin_amdgcn_perm(lo1, lo0, 0x07060302u);
}

// Writes element e of a split tensor (kind 1 or 2, scale as split_value) whose storage starts at base.
__device__ __forceinline__ void store_split(uint16_t* __restrict__ base, int64_t e, QxCplx v, int kind = 1,
                                            float scale = 1.f) {
  uint32_t hi, lo;
  split_value(kind, scale, v, hi, lo);
  uint16_t* __restrict__ c = base + split_off(e, 0);
  c[0] = (uint16_t)hi;
  c[8] = (uint16_t)lo;
  c[16] = (uint16_t)(hi >> 16);
  c[24] = (uint16_t)(lo >> 16);
}

}  // namespace qx
