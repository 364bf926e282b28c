// Seeded synthetic workloads on the device: a sparse precision matrix A_true,
// m samples x ~ N(0, A_true^{-1}) and their covariance, so that requests and
// benchmark inputs need no host-side generation.
//
// Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter and
// a 64-bit key, ten rounds of two 32x32->64-bit multiplications with the round
// constants and key increments of that paper.  Every random quantity is a pure
// function of (seed, counter), so any thread can draw any entry, and the host
// implementation in synth/philox.py gives the same words bit for bit.
//
// Recipes (counter = (c0, c1, stream, 0), key = (seed mod 2^32, seed / 2^32)):
//  * random sparse: pair (i, j), i < j, counter (j, i, 0, 0) -> words w0..w3;
//    the pair is an edge when w0 < floor(p 2^32), p = min(1, 10 / (n - 1))
//    (about ten off-diagonal nonzeros per row); value sign(w1 odd ? + : -) x
//    (0.5 + 0.5 (w2 + 0.5) 2^-32), i.e. +-U(0.5, 1); A_ii = sum_j |A_ij| + 0.1
//    (strictly diagonally dominant, hence positive definite);
//  * chain: A_ii = 1.25, A_{i,i+1} = A_{i+1,i} = -0.5;
//  * samples: z[r][c] from counter (c, r, 1, 0) by the Box-Muller transform of two
//    53-bit uniforms, u = (2^26 (w0 >> 5) + (w1 >> 6) + 1/2) 2^-53 and the same of
//    w2, w3: z = sqrt(-2 log u) cos(2 pi u'); sample r is x_r = L^{-T} z_r with
//    A_true = L L^T (Cholesky), so Cov(x) = A_true^{-1}; the rows of Y are the x_r.
#pragma clang fp contract(off)
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

struct Words {
  uint32_t w[4];
};

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c0;
    const uint64_t p1 = (uint64_t)M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  Words out;
  out.w[0] = c0;
  out.w[1] = c1;
  out.w[2] = c2;
  out.w[3] = c3;
  return out;
}

// off-diagonal entry (i, j), i != j, of the random sparse precision
__device__ __forceinline__ double sparse_entry(int64_t i, int64_t j, uint32_t k0, uint32_t k1, uint64_t thr) {
  const uint32_t lo = (uint32_t)(i < j ? i : j), hi = (uint32_t)(i < j ? j : i);
  const Words r = philox4x32_10(hi, lo, 0u, 0u, k0, k1);
  if ((uint64_t)r.w[0] >= thr) return 0.0;
  const double u = ((double)r.w[2] + 0.5) * 0x1p-32;
  const double mag = 0.5 + 0.5 * u;
  return (r.w[1] & 1u) ? mag : -mag;
}

// Lower triangle of the padded precision (np x np): zeros above the diagonal and
// the identity in the padding.  The diagonal of the random sparse recipe is
// filled by sparse_diag_kernel.
__global__ __launch_bounds__(256) void gen_lower_kernel(double* A, int64_t n, int64_t np, int kind, uint32_t k0,
                                                        uint32_t k1, uint64_t thr) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= np * np) return;
  const int64_t i = idx / np, j = idx % np;
  double v = 0.0;
  if (i >= n || j >= n) {
    v = (i == j) ? 1.0 : 0.0;
  } else if (j < i) {
    v = (kind == GEN_CHAIN) ? ((i == j + 1) ? -0.5 : 0.0) : sparse_entry(i, j, k0, k1, thr);
  } else if (j == i) {
    v = (kind == GEN_CHAIN) ? 1.25 : 0.0;
  }
  A[idx] = v;
}

// A_ii = sum_j |A_ij| + 0.1 for the random sparse recipe: one wave per row, every
// entry of the row recomputed from its counter (no strided column reads); lane l
// sums j = l, l + 64, ... in order, then a fixed butterfly.
__global__ __launch_bounds__(256) void sparse_diag_kernel(double* A, int64_t n, int64_t np, uint32_t k0, uint32_t k1,
                                                          uint64_t thr) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64)
    if (j != i) s += fabs(sparse_entry(i, j, k0, k1, thr));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) A[i * np + i] = s + 0.1;
}

// Z (mp x np): standard normals for r < m, c < n, zero in the padding
__global__ __launch_bounds__(256) void gen_normal_kernel(double* Z, int64_t m, int64_t n, int64_t mp, int64_t np,
                                                         uint32_t k0, uint32_t k1) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= mp * np) return;
  const int64_t r = idx / np, c = idx % np;
  double z = 0.0;
  if (r < m && c < n) {
    const Words w = philox4x32_10((uint32_t)c, (uint32_t)r, 1u, 0u, k0, k1);
    const double u1 = ((double)(w.w[0] >> 5) * 67108864.0 + (double)(w.w[1] >> 6) + 0.5) * 0x1p-53;
    const double u2 = ((double)(w.w[2] >> 5) * 67108864.0 + (double)(w.w[3] >> 6) + 0.5) * 0x1p-53;
    z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
  Z[idx] = z;
}

// dst (rows x cols, ld cols) <- src (ld lds)
__global__ __launch_bounds__(256) void copy_rect_kernel(const double* src, int64_t lds, double* dst, int64_t rows,
                                                        int64_t cols) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx / cols, c = idx % cols;
  dst[idx] = src[r * lds + c];
}

// per-workgroup maxima of |S_ij| over j < i < n of the padded S (its lower
// triangle: S is symmetric and only that triangle is formed)
__global__ __launch_bounds__(256) void offdiag_absmax_kernel(const double* S, int64_t n, int64_t np, double* part) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n * n; idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx / n, j = idx % n;
    if (j < i) mx = fmax(mx, fabs(S[i * np + j]));
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void max_reduce_kernel(const double* part, int count, double* out) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) mx = fmax(mx, part[i]);
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

inline unsigned blocks_for(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

int gen_precision_lower(hipStream_t stream, double* A, int64_t n, int64_t np, int kind, uint64_t seed) {
  if (n < 1 || np < n || (kind != GEN_RANDOM_SPARSE && kind != GEN_CHAIN)) return -1;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  // edge probability p = min(1, 10 / (n - 1)) as a 32-bit threshold
  uint64_t thr = (uint64_t)1 << 32;
  if (n > 11) thr = (uint64_t)floor(10.0 / (double)(n - 1) * 4294967296.0);
  hipLaunchKernelGGL(gen_lower_kernel, dim3(blocks_for(np * np)), dim3(256), 0, stream, A, n, np, kind, k0, k1, thr);
  if (hipGetLastError() != hipSuccess) return -2;
  if (kind == GEN_RANDOM_SPARSE) {
    hipLaunchKernelGGL(sparse_diag_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, A, n, np, k0, k1,
                       thr);
    if (hipGetLastError() != hipSuccess) return -2;
  }
  return 0;
}

int gen_normals(hipStream_t stream, double* Z, int64_t m, int64_t n, int64_t mp, int64_t np, uint64_t seed) {
  if (m < 1 || n < 1 || mp < m || np < n) return -1;
  hipLaunchKernelGGL(gen_normal_kernel, dim3(blocks_for(mp * np)), dim3(256), 0, stream, Z, m, n, mp, np,
                     (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int copy_rect(hipStream_t stream, const double* src, int64_t lds, double* dst, int64_t rows, int64_t cols) {
  if (rows < 1 || cols < 1 || lds < cols) return -1;
  hipLaunchKernelGGL(copy_rect_kernel, dim3(blocks_for(rows * cols)), dim3(256), 0, stream, src, lds, dst, rows,
                     cols);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int offdiag_absmax(hipStream_t stream, const double* S, int64_t n, int64_t np, double* part, double* out) {
  if (n < 1 || np < n) return -1;
  constexpr int G = 256;
  hipLaunchKernelGGL(offdiag_absmax_kernel, dim3(G), dim3(256), 0, stream, S, n, np, part);
  if (hipGetLastError() != hipSuccess) return -2;
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, stream, part, G, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
