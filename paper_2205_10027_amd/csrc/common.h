// Shared definitions for the gfx950 graphical-lasso kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace glasso {

// Every matrix the solver keeps on the device is padded to a multiple of TILE
// rows/columns; the padding block of A is the identity, so GEMM tiles never need
// bounds checks and the factor/inverse of the padded matrix is diag(L, I).
constexpr int TILE = 128;
constexpr int PASS_TILE = 64;  // tile edge of the elementwise passes

inline int64_t pad_to_tile(int64_t n) { return (n + TILE - 1) / TILE * TILE; }

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Hardware dispatches workgroup b to XCD (b mod 8).  Renumber so that every XCD
// receives a contiguous range of logical tile ids; neighbouring tiles then share
// operand panels inside one XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G >> 3, r = G & 7;
  const int x = b & 7, l = b >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Grouped row-major order over a TM x TN tile grid: runs of GM tile rows are
// walked column by column so consecutive ids reuse one B panel and GM A panels.
__device__ __forceinline__ void grouped_tile(int L, int TM, int TN, int& ti, int& tj) {
  constexpr int GM = 8;
  const int per_group = GM * TN;
  const int group = L / per_group;
  const int first = group * GM;
  const int gm = min(TM - first, GM);
  const int o = L - group * per_group;
  ti = first + o % gm;
  tj = o / gm;
}

// Tiles (ti >= tj) of the lower triangle of a T x T tile grid, enumerated in bands
// of 8 tile rows, column by column inside a band.  Band b (full) holds 64b+36
// tiles, so 32b^2 + 4b tiles precede it.
__device__ __forceinline__ void lower_tile(int L, int T, int& ti, int& tj) {
  int b = (int)((sqrt(16.0 + 128.0 * (double)L) - 4.0) / 64.0);
  while (32 * (b + 1) * (b + 1) + 4 * (b + 1) <= L) ++b;
  while (b > 0 && 32 * b * b + 4 * b > L) --b;
  int o = L - (32 * b * b + 4 * b);
  const int r0 = 8 * b;
  const int h = min(8, T - r0);
  if (o < h * r0) {
    tj = o / h;
    ti = r0 + o % h;
  } else {
    o -= h * r0;
    int c = 0;
    while (o >= h - c) {
      o -= h - c;
      ++c;
    }
    tj = r0 + c;
    ti = r0 + c + o;
  }
}

}  // namespace glasso
