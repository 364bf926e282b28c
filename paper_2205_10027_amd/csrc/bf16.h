// bf16 rounding shared by the split-operand kernels (gfx950).
#pragma once

#include <stdint.h>

#include "common.h"

namespace glasso {

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// the two-part split of an FP64 value: hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split2(double v, uint32_t& h, uint32_t& l) {
  h = bf16_bits((float)v);
  l = bf16_bits((float)(v - (double)bf16_value(h)));
}

// element (row, col) of a two-part split matrix (4 bytes per element: runs of 8 as
// 16 bytes of hi parts then 16 of lo parts), ld elements per row
__device__ __forceinline__ void store_split2(uint8_t* M, int64_t ld, int64_t row, int64_t col, double v) {
  uint32_t h, l;
  split2(v, h, l);
  uint16_t* q = reinterpret_cast<uint16_t*>(M + row * ld * 4 + (col >> 3) * 32 + (col & 7) * 2);
  q[0] = (uint16_t)h;
  q[8] = (uint16_t)l;
}

}  // namespace glasso
