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

// Factor the 128x128 diagonal block at A (lower, in place), write diag(L) to dL and
// inv(L) (zeros above the diagonal) to Dinv (ld 128).  k0 is the block's global
// column, used to report the first failing pivot through info.
__global__ __launch_bounds__(256) void leaf_potrf_inv_kernel(double* A, int64_t lda, int k0,
                                                             double* dL, double* Dinv, int* info) {
  if (*info) return;
  __shared__ double a[NB][LDL];
  __shared__ double col[NB];
  __shared__ double piv;
  const int tid = threadIdx.x;

  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e >> 7, c = e & 127;
    a[r][c] = (c <= r) ? A[(int64_t)r * lda + c] : 0.0;
  }
  __syncthreads();

  // ---- factorisation: 4 panels of 32 columns.  Thread (pr, ph) keeps row pr,
  // columns c0+16ph .. c0+16ph+15 of the current panel in registers.
  const int pr = tid >> 1, ph = tid & 1;
  int fail = -1;
#pragma unroll 1
  for (int p = 0; p < 4; ++p) {
    const int c0 = 32 * p;
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = a[pr][c0 + 16 * ph + q];
#pragma unroll
    for (int jl = 0; jl < 32; ++jl) {
      const int j = c0 + jl;
      if (fail < 0) {  // uniform: every thread reads the same pivot
        if (pr == j && ph == (jl >> 4)) {
          const double d = v[jl & 15];
          const double s = (d > 0.0 && d <= DBL_MAX) ? sqrt(d) : -1.0;
          v[jl & 15] = s;
          piv = s;
        }
        __syncthreads();
        const double ljj = piv;
        if (!(ljj > 0.0)) {
          fail = j;
        } else {
          const double rinv = 1.0 / ljj;
          if (pr > j && ph == (jl >> 4)) {
            v[jl & 15] *= rinv;
            col[pr] = v[jl & 15];
          }
          __syncthreads();
          if (pr > j) {
            const double lr = col[pr];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
              const int c = c0 + 16 * ph + q;
              if (c > j && c <= pr) v[q] -= lr * col[c];
            }
          }
        }
      }
    }
    if (fail >= 0) break;
#pragma unroll
    for (int q = 0; q < 16; ++q) a[pr][c0 + 16 * ph + q] = v[q];
    __syncthreads();
    // rank-32 update of the trailing lower triangle, 4x4 register blocks
    const int base = c0 + 32, R = NB - base;
    if (R > 0) {
      const int nb4 = R / 4;
      const int nblk = nb4 * (nb4 + 1) / 2;
      for (int e = tid; e < nblk; e += 256) {
        int bi = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((bi + 1) * (bi + 2) / 2 <= e) ++bi;
        while (bi * (bi + 1) / 2 > e) --bi;
        const int bj = e - bi * (bi + 1) / 2;
        const int r0 = base + 4 * bi, s0 = base + 4 * bj;
        double acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int w = 0; w < 4; ++w) acc[u][w] = 0.0;
#pragma unroll 2
        for (int k = c0; k < c0 + 32; ++k) {
          double x[4], y[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            x[u] = a[r0 + u][k];
            y[u] = a[s0 + u][k];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[u][w] += x[u] * y[w];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int w = 0; w < 4; ++w)
            if (s0 + w <= r0 + u) a[r0 + u][s0 + w] -= acc[u][w];
      }
      __syncthreads();
    }
  }
  if (fail >= 0) {
    if (tid == 0) *info = k0 + fail + 1;
    return;
  }

  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e >> 7, c = e & 127;
    if (c <= r) A[(int64_t)r * lda + c] = a[r][c];
  }
  if (tid < NB) dL[tid] = a[tid][tid];

  // ---- in-place inverse of the lower-triangular block, last column first:
  // column j of inv(L) = -(1/L_jj) * inv(L)[j+1:, j+1:] * L[j+1:, j].
  for (int j = NB - 1; j >= 0; --j) {
    if (tid < NB && tid > j) col[tid] = a[tid][j];
    __syncthreads();
    const double dinv = 1.0 / a[j][j];
    const int i = j + 1 + (tid >> 1);
    double s = 0.0;
    if (i < NB) {
      for (int k = j + 1 + (tid & 1); k <= i; k += 2) s += a[i][k] * col[k];
    }
    s += __shfl_xor(s, 1);
    __syncthreads();
    if (i < NB && (tid & 1) == 0) a[i][j] = -dinv * s;
    if (tid == 0) a[j][j] = dinv;
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e >> 7, c = e & 127;
    Dinv[e] = (c <= r) ? a[r][c] : 0.0;
  }
}

// Place the stored diagonal-block inverses on the diagonal of L.
__global__ __launch_bounds__(256) void copy_diag_blocks_kernel(double* L, int64_t ld, const double* Dinv,
                                                               const int* abort_flag) {
  if (abort_flag && *abort_flag) return;
  const int b = blockIdx.x;
  const double* src = Dinv + (int64_t)b * NB * NB;
  double* dst = L + (int64_t)b * NB * (ld + 1);
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e >> 7, c = e & 127;
    dst[(int64_t)r * ld + c] = src[e];
  }
}

}  // namespace

int potrf_lower(hipStream_t stream, double* A, int64_t lda, int n, double* dL, double* Dinv, int* info) {
  if (n % NB) return -1;
  int rc = 0;
  for (int K0 = 0; K0 < n && rc == 0; K0 += OUTER) {
    const int K1 = min(K0 + OUTER, n);
    for (int k = K0; k < K1 && rc == 0; k += NB) {
      double* Akk = A + (int64_t)k * lda + k;
      hipLaunchKernelGGL(leaf_potrf_inv_kernel, dim3(1), dim3(256), 0, stream, Akk, lda, k, dL + k,
                         Dinv + (int64_t)(k / NB) * NB * NB, info);
      if (hipGetLastError() != hipSuccess) return -2;
      const int rest = n - k - NB;
      if (rest > 0) {
        // panel below the block: A21 <- A21 * inv(L11)^T (in place; one tile column)
        double* A21 = A + (int64_t)(k + NB) * lda + k;
        rc = gemm_f64(stream, 0, 0, rest, NB, NB, 1.0, A21, lda, Dinv + (int64_t)(k / NB) * NB * NB, NB,
                      0.0, A21, lda, 0, 0, 2, info);
        if (rc) return rc;
      }
      if (k + NB < K1) {
        // update of the remaining columns of the outer panel
        const double* Pk = A + (int64_t)(k + NB) * lda + k;
        rc = gemm_f64(stream, 0, 0, rest, K1 - k - NB, NB, -1.0, Pk, lda, Pk, lda, 1.0,
                      A + (int64_t)(k + NB) * lda + (k + NB), lda, 0, 0, 0, info);
        if (rc) return rc;
      }
    }
    if (K1 < n) {
      // trailing lower triangle: A22 -= L21 L21^T with K = panel width
      const double* L21 = A + (int64_t)K1 * lda + K0;
      rc = gemm_f64(stream, 0, 0, n - K1, n - K1, K1 - K0, -1.0, L21, lda, L21, lda, 1.0,
                    A + (int64_t)K1 * lda + K1, lda, 1, 0, 0, info);
    }
  }
  return rc;
}

int trtri_lower(hipStream_t stream, double* L, int64_t ld, int n, const double* Dinv, double* tmp,
                const int* abort_flag) {
  if (n % NB) return -1;
  const int nblk = n / NB;
  hipLaunchKernelGGL(copy_diag_blocks_kernel, dim3(nblk), dim3(256), 0, stream, L, ld, Dinv, abort_flag);
  if (hipGetLastError() != hipSuccess) return -2;
  // doubling: at block size s, each group [T11 0; T21 T22] of size 2s gets
  // X21 = -inv(T22) * T21 * inv(T11)
  for (int64_t s = NB; s < n; s *= 2) {
    const int64_t gstride = 2 * s * (ld + 1);
    const int full = (int)(n / (2 * s));
    int rc;
    if (full > 0) {
      rc = gemm_f64(stream, 0, 1, (int)s, (int)s, (int)s, 1.0, L + s * ld, ld, L, ld, 0.0, tmp, s, 0, 0, 1,
                    abort_flag, full, gstride, gstride, s * s);
      if (rc) return rc;
      rc = gemm_f64(stream, 0, 1, (int)s, (int)s, (int)s, -1.0, L + s * (ld + 1), ld, tmp, s, 0.0, L + s * ld,
                    ld, 0, 1, 0, abort_flag, full, gstride, s * s, gstride);
      if (rc) return rc;
    }
    const int64_t base = (int64_t)full * 2 * s;
    const int64_t n2 = n - base - s;
    if (n2 > 0) {
      rc = gemm_f64(stream, 0, 1, (int)n2, (int)s, (int)s, 1.0, L + (base + s) * ld + base, ld,
                    L + base * (ld + 1), ld, 0.0, tmp, s, 0, 0, 1, abort_flag);
      if (rc) return rc;
      rc = gemm_f64(stream, 0, 1, (int)n2, (int)s, (int)n2, -1.0, L + (base + s) * (ld + 1), ld, tmp, s, 0.0,
                    L + (base + s) * ld + base, ld, 0, 1, 0, abort_flag);
      if (rc) return rc;
    }
  }
  return 0;
}

int lauum_lower(hipStream_t stream, const double* V, int64_t ldv, double* W, int64_t ldw, int n) {
  // W = V^T V: op(A) = V^T is upper triangular, op(B) = V lower; tile (i, j) sums k >= i.
  return gemm_f64(stream, 1, 1, n, n, n, 1.0, V, ldv, V, ldv, 0.0, W, ldw, 1, 2, 1, nullptr);
}

}  // namespace glasso
