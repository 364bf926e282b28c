// Blocked Cholesky factorisation, triangular inverse and LAUUM product for the
// FP64 path (gfx950).  W = A^{-1} = L^{-T} L^{-1} gives the gradient S - W
// (eq. grad_hessian); the factor of every line-search trial decides positive
// definiteness and gives log det (condition t_cond_pd).
//
// Layout: row-major, padded to multiples of 128; only lower triangles are read.
// The bulk of the flops runs in gemm_f64 (MFMA); the 128x128 diagonal blocks are
// factored and inverted by one workgroup in LDS.
#include <float.h>

#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

constexpr int NB = 128;        // leaf block (= GEMM tile)
constexpr int LDL = NB + 1;    // LDS row stride of the leaf
constexpr int OUTER = 1024;    // outer panel width of the two-level Cholesky

constexpr int PW = 32;  // panel width inside the leaf

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
template <bool NN, bool LOWA, bool LOWB>
__device__ __forceinline__ v4d mfma_block(const double (*a)[LDL], int ar, int ac, int br, int bc, int K, v4d acc,
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

// ---- in-LDS inverse of a lower-triangular 128x128 block (upper triangle = scratch)
//
// Stage 1: wave w inverts the 32x32 diagonal block w (lane c computes column c by
// forward substitution).  Stage 2 doubles the inverted block size: for each group
// [T11 0; T21 T22] of size 2S with T11, T22 already inverted,
//   tmp = T21 inv(T11)  (stored transposed in the free upper triangle),
//   X21 = -inv(T22) tmp (written over T21),
// as 16x16 MFMA blocks spread over the four waves.
template <int S>
__device__ __forceinline__ void trtri_level(double (*a)[LDL], int tid) {
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

__device__ void lds_trtri128(double (*a)[LDL], int tid) {
  const int lane = tid & 63, wave = tid >> 6;
  if (lane < PW) {
    const int o = PW * wave;
    double x[PW];
#pragma unroll
    for (int i = 0; i < PW; ++i) {
      double s = (i == lane) ? 1.0 : 0.0;
      // Row i's loads may not start before x[i-2] exists: without this ordering the
      // compiler hoists all 528 loads of the block and spills.
      int rb = (o + i) * LDL + o;
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
  trtri_level<32>(a, tid);
  trtri_level<64>(a, tid);
}

// Factor the 128x128 diagonal block at A (lower, in place), write diag(L) to dL and
// inv(L) (zeros above the diagonal) to Dinv (ld 128).  k0 is the block's global
// column, used to report the first failing pivot through info.
//
// Four panels of 32 columns.  For a panel starting at c0, every wave holds the
// 32x32 diagonal block in lanes 0..31 (row c0+lane, one register per column) and
// factors it redundantly: the pivot comes from readlane, the multipliers of the
// block rows are broadcast through the wave's own LDS row.  Lanes 32..63 of the
// waves hold the rows below the block and are eliminated in the same steps (the
// triangular solve of the panel).  All 4 waves then apply the rank-32 update to
// the trailing lower triangle.  Elements above the diagonal carry garbage and are
// never read as data.
__global__ __launch_bounds__(256) void leaf_potrf_inv_kernel(double* A, int64_t lda, int k0,
                                                             double* dL, double* Dinv, int* info,
                                                             FactorBatch fb) {
  // problem blockIdx.y of the batch
  A += blockIdx.y * fb.sA;
  dL += blockIdx.y * fb.sdL;
  Dinv += blockIdx.y * fb.sDinv;
  info += blockIdx.y;
  if (*info) return;
  __shared__ double a[NB][LDL];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // 32 independent 16-byte loads per thread (a wave reads 4 rows of 1 KB)
#pragma unroll 8
  for (int i = 0; i < NB * NB / 512; ++i) {
    const int e = 2 * (tid + 256 * i);
    const int r = e >> 7, c = e & 127;
    const double2 x = *reinterpret_cast<const double2*>(A + (int64_t)r * lda + c);
    a[r][c] = (c <= r) ? x.x : 0.0;
    a[r][c + 1] = (c + 1 <= r) ? x.y : 0.0;
  }
  __syncthreads();

  int fail = -1;  // identical in every wave: all waves factor the same block
#pragma unroll 1
  for (int p = 0; p < NB / PW; ++p) {
    const int c0 = PW * p;
    const int row = (lane < PW) ? c0 + lane : c0 + PW + wave * PW + (lane - PW);
    const bool valid = row < NB;
    double v[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) v[q] = valid ? a[row][c0 + q] : 0.0;
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      const double piv = lane_bcast(v[j], j);
      const bool ok = (piv > 0.0) && (piv <= DBL_MAX);
      if (!ok && fail < 0) fail = c0 + j;
      const double r = rsqrt(ok ? piv : 1.0);
      const double m = v[j] * r;  // lane j: sqrt(piv); rows below: multipliers
      v[j] = m;
      // the multipliers of the block rows are uniform values: broadcast each one
      // from its lane with readlane and update every later column
#pragma unroll
      for (int c = j + 1; c < PW; ++c) v[c] -= m * lane_bcast(m, c);
    }
    if (fail >= 0) break;
    if (valid && (lane >= PW || wave == 0)) {
#pragma unroll
      for (int q = 0; q < PW; ++q) a[row][c0 + q] = v[q];
    }
    __syncthreads();
    // rank-32 update of the trailing lower triangle in 16x16 MFMA blocks
    const int base = c0 + PW, R = NB - base;
    if (R > 0) {
      const int nb16 = R / 16;
      const int nblk = nb16 * (nb16 + 1) / 2;
      for (int job = wave; job < nblk; job += 4) {
        int bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= job) ++bi;
        const int bj = job - bi * (bi + 1) / 2;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        acc = mfma_block<false, false, false>(a, base + 16 * bi, c0, base + 16 * bj, c0, PW, acc, lane);
        for_block(acc, lane, [&](int r, int c, double v) { a[base + 16 * bi + r][base + 16 * bj + c] -= v; });
      }
      __syncthreads();
    }
  }
  if (fail >= 0) {
    if (tid == 0) *info = k0 + fail + 1;
    return;
  }

#pragma unroll 8
  for (int i = 0; i < NB * NB / 256; ++i) {
    const int e = tid + 256 * i;
    const int r = e >> 7, c = e & 127;
    if (c <= r) A[(int64_t)r * lda + c] = a[r][c];
  }
  if (tid < NB) dL[tid] = a[tid][tid];
  __syncthreads();
  lds_trtri128(a, tid);
#pragma unroll 8
  for (int i = 0; i < NB * NB / 256; ++i) {
    const int e = tid + 256 * i;
    const int r = e >> 7, c = e & 127;
    Dinv[e] = (c <= r) ? a[r][c] : 0.0;
  }
}

// Place the stored diagonal-block inverses on the diagonal of L.
__global__ __launch_bounds__(256) void copy_diag_blocks_kernel(double* L, int64_t ld, const double* Dinv,
                                                               const int* abort_flag, FactorBatch fb) {
  if (abort_flag && abort_flag[blockIdx.y]) return;
  const int b = blockIdx.x;
  const double* src = Dinv + blockIdx.y * fb.sDinv + (int64_t)b * NB * NB;
  double* dst = L + blockIdx.y * fb.sA + (int64_t)b * NB * (ld + 1);
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e >> 7, c = e & 127;
    dst[(int64_t)r * ld + c] = src[e];
  }
}

}  // namespace

int potrf_lower(hipStream_t stream, double* A, int64_t lda, int n, double* dL, double* Dinv, int* info,
                const FactorBatch& fb) {
  if (n % NB) return -1;
  if (fb.count <= 0) return 0;
  ZBatch zA;  // operands and output inside the factored matrix
  zA.count = fb.count;
  zA.sA = zA.sB = zA.sC = fb.sA;
  ZBatch zT = zA;  // triangular solve: B operand is the diagonal-block inverse
  zT.sB = fb.sDinv;
  int rc = 0;
  for (int K0 = 0; K0 < n && rc == 0; K0 += OUTER) {
    const int K1 = min(K0 + OUTER, n);
    for (int k = K0; k < K1 && rc == 0; k += NB) {
      double* Akk = A + (int64_t)k * lda + k;
      hipLaunchKernelGGL(leaf_potrf_inv_kernel, dim3(1, fb.count), dim3(256), 0, stream, Akk, lda, k, dL + k,
                         Dinv + (int64_t)(k / NB) * NB * NB, info, fb);
      if (hipGetLastError() != hipSuccess) return -2;
      const int rest = n - k - NB;
      if (rest > 0) {
        // panel below the block: A21 <- A21 * inv(L11)^T (in place; one tile column)
        double* A21 = A + (int64_t)(k + NB) * lda + k;
        rc = gemm_f64(stream, 0, 0, rest, NB, NB, 1.0, A21, lda, Dinv + (int64_t)(k / NB) * NB * NB, NB,
                      0.0, A21, lda, 0, 0, 2, info, 1, 0, 0, 0, 0, zT, /*in_place=*/1);
        if (rc) return rc;
      }
      if (k + NB < K1) {
        // update of the remaining columns of the outer panel
        const double* Pk = A + (int64_t)(k + NB) * lda + k;
        rc = gemm_f64(stream, 0, 0, rest, K1 - k - NB, NB, -1.0, Pk, lda, Pk, lda, 1.0,
                      A + (int64_t)(k + NB) * lda + (k + NB), lda, 0, 0, 0, info, 1, 0, 0, 0, 0, zA);
        if (rc) return rc;
      }
    }
    if (K1 < n) {
      // trailing lower triangle: A22 -= L21 L21^T with K = panel width
      const double* L21 = A + (int64_t)K1 * lda + K0;
      rc = gemm_f64(stream, 0, 0, n - K1, n - K1, K1 - K0, -1.0, L21, lda, L21, lda, 1.0,
                    A + (int64_t)K1 * lda + K1, lda, 1, 0, 0, info, 1, 0, 0, 0, 0, zA);
    }
  }
  return rc;
}

int trtri_lower(hipStream_t stream, double* L, int64_t ld, int n, const double* Dinv, double* tmp,
                const int* abort_flag, const FactorBatch& fb, int64_t sTmp) {
  if (n % NB) return -1;
  if (fb.count <= 0) return 0;
  const int nblk = n / NB;
  hipLaunchKernelGGL(copy_diag_blocks_kernel, dim3(nblk, fb.count), dim3(256), 0, stream, L, ld, Dinv, abort_flag,
                     fb);
  if (hipGetLastError() != hipSuccess) return -2;
  ZBatch z1;  // tmp = T21 inv(T11)
  z1.count = fb.count;
  z1.sA = fb.sA;
  z1.sB = fb.sA;
  z1.sC = sTmp;
  ZBatch z2;  // T21 = -inv(T22) tmp
  z2.count = fb.count;
  z2.sA = fb.sA;
  z2.sB = sTmp;
  z2.sC = fb.sA;
  // doubling: at block size s, each group [T11 0; T21 T22] of size 2s gets
  // X21 = -inv(T22) * T21 * inv(T11)
  for (int64_t s = NB; s < n; s *= 2) {
    const int64_t gstride = 2 * s * (ld + 1);
    const int full = (int)(n / (2 * s));
    int rc;
    if (full > 0) {
      rc = gemm_f64(stream, 0, 1, (int)s, (int)s, (int)s, 1.0, L + s * ld, ld, L, ld, 0.0, tmp, s, 0, 0, 1,
                    abort_flag, full, gstride, gstride, s * s, 0, z1);
      if (rc) return rc;
      rc = gemm_f64(stream, 0, 1, (int)s, (int)s, (int)s, -1.0, L + s * (ld + 1), ld, tmp, s, 0.0, L + s * ld,
                    ld, 0, 1, 0, abort_flag, full, gstride, s * s, gstride, 0, z2);
      if (rc) return rc;
    }
    const int64_t base = (int64_t)full * 2 * s;
    const int64_t n2 = n - base - s;
    if (n2 > 0) {
      rc = gemm_f64(stream, 0, 1, (int)n2, (int)s, (int)s, 1.0, L + (base + s) * ld + base, ld,
                    L + base * (ld + 1), ld, 0.0, tmp, s, 0, 0, 1, abort_flag, 1, 0, 0, 0, 0, z1);
      if (rc) return rc;
      rc = gemm_f64(stream, 0, 1, (int)n2, (int)s, (int)n2, -1.0, L + (base + s) * (ld + 1), ld, tmp, s, 0.0,
                    L + (base + s) * ld + base, ld, 0, 1, 0, abort_flag, 1, 0, 0, 0, 0, z2);
      if (rc) return rc;
    }
  }
  return 0;
}

int lauum_lower(hipStream_t stream, const double* V, int64_t ldv, double* W, int64_t ldw, int n,
                const int* abort_flag, const FactorBatch& fb, int64_t sW) {
  // W = V^T V: op(A) = V^T is upper triangular, op(B) = V lower; tile (i, j) sums k >= i.
  ZBatch z;
  z.count = fb.count;
  z.sA = z.sB = fb.sA;
  z.sC = sW;
  return gemm_f64(stream, 1, 1, n, n, n, 1.0, V, ldv, V, ldv, 0.0, W, ldw, 1, 2, 1, abort_flag, 1, 0, 0, 0, 0, z);
}

}  // namespace glasso
