// Factorisation and inversion of one diagonal block held in LDS by one
// workgroup of 256 threads (4 wave64s), for block edges NB = 64 and 128.  Used by
// the blocked Cholesky (NB = 128 leaf blocks) and the persistent small-problem
// solver (NB = 64: the whole matrix).
#pragma once

#include <float.h>

#include "common.h"

namespace glasso {

namespace {

constexpr int PW = 32;  // edge of the diagonal blocks inverted in the first stage of lds_trtri

// 1/sqrt(x) for a positive normal x: the hardware estimate refined by one
// third-order step, t (1 + e/2 + 3e^2/8) with e = 1 - x t^2 (no special cases)
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double t = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * t, t, 1.0);
  return fma(t * e, fma(e, 0.375, 0.5), t);
}

// broadcast a double from a wave-uniform lane
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// ---- small FP64 MFMA products on LDS-resident operands
//
// One 16x16 output block per call: acc += A B over k in [0, K), A element (m, k)
// at a[ar + m][ac + k]; B element (k, n) at a[br + n][bc + k] (NT: rows of B^T)
// or at a[br + k][bc + n] (NN).  Lane l supplies A[l%16][k + l/16] and
// B[k + l/16][l%16]; D[i][j] lands in lane j + 16 (i%4), register i/4.
// Optional masks zero A where k > m (A lower) and B where k < n (B lower), in
// operand-local indices (mask_a/mask_b give the offsets of the block in the
// triangular operand).
template <bool NN, bool LOWA, bool LOWB, int LD>
__device__ __forceinline__ v4d mfma_block(const double (*a)[LD], int ar, int ac, int br, int bc, int K, v4d acc,
                                          int lane, int ma = 0, int mb = 0) {
  const int i = lane & 15, kk = lane >> 4;
#pragma unroll 4
  for (int k = 0; k < K; k += 4) {
    double x = a[ar + i][ac + k + kk];
    double y = NN ? a[br + k + kk][bc + i] : a[br + i][bc + k + kk];
    if (LOWA && (k + kk > ma + i)) x = 0.0;
    if (LOWB && (k + kk < mb + i)) y = 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
  }
  return acc;
}

// element (4r + lane/16, lane%16) of a 16x16 MFMA block is acc[r]
template <typename F>
__device__ __forceinline__ void for_block(v4d acc, int lane, F f) {
#pragma unroll
  for (int r = 0; r < 4; ++r) f(4 * r + (lane >> 4), lane & 15, acc[r]);
}

// ---- in-LDS inverse of a lower-triangular NB x NB block (upper triangle = scratch)
//
// Stage 1: wave w inverts the 32x32 diagonal block w (lane c computes column c by
// forward substitution).  Stage 2 doubles the inverted block size: for each group
// [T11 0; T21 T22] of size 2S with T11, T22 already inverted,
//   tmp = T21 inv(T11)  (stored transposed in the free upper triangle),
//   X21 = -inv(T22) tmp (written over T21),
// as 16x16 MFMA blocks spread over the four waves.
template <int S, int NB>
__device__ __forceinline__ void trtri_level(double (*a)[NB + 1], int tid) {
  constexpr int NBS = S / 16;                 // 16-blocks per edge
  constexpr int GROUPS = NB / (2 * S);
  constexpr int JOBS = GROUPS * NBS * NBS;    // output blocks per product
  const int lane = tid & 63, wave = tid >> 6;
  // tmp = T21 inv(T11): block (bi, bj) sums k from 16 bj (inv(T11) is lower)
  for (int job = wave; job < JOBS; job += 4) {
    const int g = job / (NBS * NBS), bi = (job / NBS) % NBS, bj = job % NBS;
    const int o = g * 2 * S;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    const int k0 = 16 * bj;
    acc = mfma_block<true, false, true>(a, o + S + 16 * bi, o + k0, o + k0, o + 16 * bj, S - k0, acc, lane, 0, 0);
    for_block(acc, lane, [&](int r, int c, double v) { a[o + 16 * bj + c][o + S + 16 * bi + r] = v; });
  }
  __syncthreads();
  // X21 = -inv(T22) tmp: block (bi, bj) sums k up to 16 bi + 15 (inv(T22) is lower)
  for (int job = wave; job < JOBS; job += 4) {
    const int g = job / (NBS * NBS), bi = (job / NBS) % NBS, bj = job % NBS;
    const int o = g * 2 * S;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    acc = mfma_block<false, true, false>(a, o + S + 16 * bi, o + S, o + 16 * bj, o + S, 16 * (bi + 1), acc, lane,
                                         16 * bi, 0);
    for_block(acc, lane, [&](int r, int c, double v) { a[o + S + 16 * bi + r][o + 16 * bj + c] = -v; });
  }
  __syncthreads();
}

template <int NB>
__device__ void lds_trtri(double (*a)[NB + 1], int tid) {
  static_assert(NB == 64 || NB == 128, "block edge");
  const int lane = tid & 63, wave = tid >> 6;
  if (lane < PW && PW * wave < NB) {
    const int o = PW * wave;
    double x[PW];
#pragma unroll
    for (int i = 0; i < PW; ++i) {
      double s = (i == lane) ? 1.0 : 0.0;
      // Row i's loads may not start before x[i-2] exists: without this ordering the
      // compiler hoists all 528 loads of the block and spills.
      int rb = (o + i) * (NB + 1) + o;
      if (i >= 2) asm volatile("" : "+v"(rb) : "v"(x[i - 2]));
      const double* arow = &a[0][0] + rb;
#pragma unroll
      for (int k = 0; k < i; ++k) s -= arow[k] * x[k];
      x[i] = s / arow[i];
    }
    // x[i] = 0 for i < lane: only the lower part of column `lane` is written
#pragma unroll
    for (int i = 0; i < PW; ++i)
      if (i >= lane) a[o + i][o + lane] = x[i];
  }
  __syncthreads();
  trtri_level<32, NB>(a, tid);
  if (NB == 128) trtri_level<64, NB>(a, tid);
}

// Cholesky of the NB x NB lower triangle in LDS, in place.  Returns the first
// failing pivot (non-positive or NaN) or -1; the value is identical in every
// thread, and on failure the block is left partially factored.
//
// Panels of PF = 16 columns (one column of 16x16 blocks).  The lower triangle's
// 16x16 blocks live in the waves' MFMA accumulators between panels: block k of
// the list "column NB/16 - 1 first, then leftwards, rows top-down inside a
// column" belongs to wave k % 4, slot k / 4, so the blocks still to be updated
// after any panel are a prefix of the list and spread evenly over the waves.
// For panel p:
//   1. the owners write block column p to LDS;
//   2. every wave factors the panel redundantly: the 16x16 diagonal block in lanes
//      0..15 (row c0+lane, one register per column), column j of its rows broadcast
//      with readlane (its first entry is the pivot); lanes 16..63 hold the rows
//      below (48 per wave) and are eliminated in the same steps.  The factored panel
//      goes to LDS;
//   3. each wave subtracts the panel's rank-16 product from its own blocks right of
//      the panel, four independent MFMAs per block, operands from LDS.  (Spreading
//      these MFMAs over the next panel's pivot steps does not hide them: the pivot
//      chain then ran twice as long.)
// The broadcasts grow with the square of the panel width, the update rounds only
// linearly with the number of panels, which is why the panels are narrow.
// Elements above the diagonal are never read as data.
// `pre` (optional) runs after the blocks are in the accumulators and before the
// first panel, with the LDS block free for its own staging: it may subtract further
// products from the accumulators (the leaf step's left-looking updates); block
// column 0 then goes back to LDS from the accumulators like every later one.
constexpr int PF = 16;

struct NoPre {
  template <int SL>
  __device__ void operator()(v4d (&)[SL], const int (&)[SL], const int (&)[SL]) const {}
};

template <int NB, typename Pre = NoPre>
__device__ int lds_potrf(double (*a)[NB + 1], int tid, Pre pre = Pre()) {
  constexpr bool kPre = !__is_same(Pre, NoPre);
  constexpr int NBB = NB / 16;               // 16x16 blocks per edge
  constexpr int NBLK = NBB * (NBB + 1) / 2;  // blocks of the lower triangle
  constexpr int SLOTS = (NBLK + 3) / 4;      // blocks per wave
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  int bi[SLOTS], bj[SLOTS];
  v4d acc[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int k = 4 * s + wave;
    int c = NBB - 1, start = 0;
    while (c >= 0 && k >= start + (NBB - c)) {
      start += NBB - c;
      --c;
    }
    bj[s] = (k < NBLK) ? c : -1;
    bi[s] = (k < NBLK) ? c + (k - start) : 0;
    // element (4r + lane/16, lane%16) of a block is register r (FP64 MFMA output layout)
    if (bj[s] >= 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[s][r] = a[16 * bi[s] + 4 * r + lk][16 * bj[s] + li];
    }
  }
  if (kPre) {
    __syncthreads();  // every wave has its blocks: the LDS block is free
    pre(acc, bi, bj);
  }
  int fail = -1;
#pragma unroll 1
  for (int p = 0; p < NBB; ++p) {
    const int c0 = PF * p;
    if (p > 0 || kPre) {
#pragma unroll
      for (int s = 0; s < SLOTS; ++s)
        if (bj[s] == p) for_block(acc[s], lane, [&](int r, int c, double v) { a[16 * bi[s] + r][c0 + c] = v; });
    }
    __syncthreads();
    const int row = (lane < PF) ? c0 + lane : c0 + PF + wave * (64 - PF) + (lane - PF);
    const bool valid = row < NB;
    const int lrow = valid ? row : NB - 1;  // in-bounds row for the unconditional loads
    double v[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const double t = a[lrow][c0 + q];
      v[q] = valid ? t : 0.0;
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      // column j of the block rows, unscaled, as uniform values (readlane): they do
      // not wait for the pivot's square root
      double u[PF];
#pragma unroll
      for (int c = j; c < PF; ++c) u[c] = lane_bcast(v[j], c);
      // a pivot that is not positive and finite gives garbage from here on (at
      // least a diagonal entry that is not either); the panel is checked below
      const double piv = u[j];
      const double r = rsqrt_pos(piv);
      // L[row][j] L[c][j] = v[j] u[c] / piv
      const double y = v[j] * (r * r);
      v[j] = v[j] * r;  // lane j: sqrt(piv); rows below: L[row][j]
#pragma unroll
      for (int c = j + 1; c < PF; ++c) v[c] -= y * u[c];
    }
    if (valid && (lane >= PF || wave == 0)) {
#pragma unroll
      for (int q = 0; q < PF; ++q) a[row][c0 + q] = v[q];
    }
    __syncthreads();
    {
      // the panel's first pivot that is not positive and finite is the first of its
      // diagonal entries sqrt(piv) that is not (rsqrt of a negative, zero, infinite
      // or NaN pivot gives NaN): one check per panel, not a branch in every step
      const double d = a[c0 + (lane & 15)][c0 + (lane & 15)];
      const uint64_t bad = __ballot(!(d > 0.0 && d <= DBL_MAX));
      if (bad) {
        fail = c0 + __builtin_ctzll(bad);
        break;
      }
    }
    // blocks right of the panel: acc -= L[bi rows][panel] L[bj rows][panel]^T
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (bj[s] > p) {
#pragma unroll
        for (int k = 0; k < PF; k += 4) {
          const double x = a[16 * bi[s] + li][c0 + k + lk];
          const double y = a[16 * bj[s] + li][c0 + k + lk];
          acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x, y, acc[s], 0, 0, 0);
        }
      }
    }
  }
  return fail;
}

}  // namespace

}  // namespace glasso
