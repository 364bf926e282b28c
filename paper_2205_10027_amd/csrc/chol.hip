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
#include "leaf.h"

namespace glasso {

namespace {

constexpr int NB = 128;        // leaf block (= GEMM tile)
constexpr int LDL = NB + 1;    // LDS row stride of the leaf
constexpr int OUTER = 1024;    // outer panel width of the two-level Cholesky

// One step of the blocked Cholesky: the 128-column block whose diagonal block is at
// A, with `rest` rows of the panel below it (a multiple of 64).
//
// Every workgroup factors (lds_potrf) and inverts (lds_trtri) the diagonal block in
// LDS; all of them compute identical values.  Workgroup 0 writes diag(L) to dL,
// inv(L11) to Dinv (ld 128, zeros above the diagonal) and the strict lower part of
// L11 transposed into the strict upper triangle of the block: the lower triangle is
// still being read by the other workgroups, so place_diag_factor moves L11 into
// place after the whole factorisation.  Workgroup 1 + q solves rows 64q .. 64q + 63
// of the panel below, L21 = A21 inv(L11)^T, in place: it owns those rows entirely.
// k0 is the block's global column, used to report the first failing pivot.
__global__ __launch_bounds__(256) void leaf_potrf_inv_kernel(double* A, int64_t lda, int k0, int rest,
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

  const int fail = lds_potrf<NB>(a, tid);
  if (fail >= 0) {
    if (blockIdx.x == 0 && tid == 0) *info = k0 + fail + 1;
    return;
  }
  if (blockIdx.x == 0) {
#pragma unroll 8
    for (int i = 0; i < NB * NB / 256; ++i) {
      const int e = tid + 256 * i;
      const int r = e >> 7, c = e & 127;
      if (c < r) A[(int64_t)c * lda + r] = a[r][c];
    }
    if (tid < NB) dL[tid] = a[tid][tid];
  }
  __syncthreads();
  lds_trtri<NB>(a, tid);
  if (blockIdx.x == 0) {
#pragma unroll 8
    for (int i = 0; i < NB * NB / 256; ++i) {
      const int e = tid + 256 * i;
      const int r = e >> 7, c = e & 127;
      Dinv[e] = (c <= r) ? a[r][c] : 0.0;
    }
    return;
  }
  if (rest <= 0) return;
  // rows 64q .. 64q + 63 below the block; wave w takes 16 of them.  A operand of
  // k-step s: R[16w + lane%16][4s + lane/16] (v_mfma_f64_16x16x4f64 A layout);
  // B operand inv(L11)^T (k, c) = inv(L11)[c][k], zero for k > c (the upper
  // triangle of a is scratch).
  double* R = A + (int64_t)(NB + 64 * (blockIdx.x - 1)) * lda;
  const double* Rw = R + (int64_t)(16 * wave + (lane & 15)) * lda + (lane >> 4);
  double af[NB / 4];
#pragma unroll
  for (int s = 0; s < NB / 4; ++s) af[s] = Rw[4 * s];
  v4d acc[8];
#pragma unroll
  for (int cb = 0; cb < 8; ++cb) acc[cb] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < NB / 4; ++s) {
#pragma unroll
    for (int cb = s / 4; cb < 8; ++cb) {
      const int c = 16 * cb + (lane & 15), k = 4 * s + (lane >> 4);
      const double y = (k <= c) ? a[c][k] : 0.0;
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s], y, acc[cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 8; ++cb)
    for_block(acc[cb], lane, [&](int r, int c, double v) { R[(int64_t)(16 * wave + r) * lda + 16 * cb + c] = v; });
}

// After the factorisation: the strict lower part of every 128x128 diagonal block
// from its transposed copy in the strict upper triangle, the diagonal from dL.
__global__ __launch_bounds__(256) void place_diag_factor_kernel(double* A, int64_t lda, const double* dL,
                                                                const int* info, FactorBatch fb) {
  if (info[blockIdx.y]) return;
  double* D = A + blockIdx.y * fb.sA + (int64_t)blockIdx.x * NB * (lda + 1);
  const double* d = dL + blockIdx.y * fb.sdL + (int64_t)blockIdx.x * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e >> 7, c = e & 127;
    if (c < r)
      D[(int64_t)r * lda + c] = D[(int64_t)c * lda + r];
    else if (c == r)
      D[(int64_t)r * lda + r] = d[r];
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
  int rc = 0;
  for (int K0 = 0; K0 < n && rc == 0; K0 += OUTER) {
    const int K1 = min(K0 + OUTER, n);
    for (int k = K0; k < K1 && rc == 0; k += NB) {
      // factor + invert the diagonal block and solve the panel below it (L21 = A21 inv(L11)^T)
      double* Akk = A + (int64_t)k * lda + k;
      const int rest = n - k - NB;
      hipLaunchKernelGGL(leaf_potrf_inv_kernel, dim3(1 + rest / 64, fb.count), dim3(256), 0, stream, Akk, lda, k,
                         rest, dL + k, Dinv + (int64_t)(k / NB) * NB * NB, info, fb);
      if (hipGetLastError() != hipSuccess) return -2;
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
  if (rc) return rc;
  hipLaunchKernelGGL(place_diag_factor_kernel, dim3(n / NB, fb.count), dim3(256), 0, stream, A, lda, dL, info, fb);
  return hipGetLastError() == hipSuccess ? 0 : -2;
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
