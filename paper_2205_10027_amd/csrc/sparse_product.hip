// The preconditioned product P = A Z A (eq. b) on the free set, for iterates with
// short rows.
//
// The trial point (eq. d_sol) reads P only where the free-set mask M is set, and
// only in the lower triangle (P is symmetric).  When every row of the iterate A
// holds at most SPARSE_KA nonzeros and every row of M at most SPARSE_KM entries
// at or left of the diagonal, each needed entry is the bilinear form
//   P_ij = sum_{k in nz(A_j)} ( sum_{l in nz(A_i)} A_il Z_lk ) A_jk,
// summed in the order the dense GEMM pair uses (X = A Z first, then X A), in
// FP64.  Its cost is |M| * |nz(A_i)| * |nz(A_j)| gathers instead of 2 np^3 flops.
// A problem whose rows are longer keeps the dense pair: the decision is taken on
// the device per problem and product, so a captured graph covers both cases.
//
// Steps (all per problem of the batch, problems with skip != 0 untouched):
//   sparse_rows_kernel    one wave per row: column lists of A (with values) and of
//                         the lower part of M, and their lengths;
//   sparse_decide_kernel  one workgroup per problem: dense[b] = some row too long,
//                         dskip[b] = the dense pair's skip flag, and the choice
//                         into the problem's scalar slot SC_DENSE_PRODUCT;
//   sparse_product_kernel one wave per row i, one lane per entry (i, j) of M.
// Z is read as FP64, or from its hi + lo bf16 split (the BF16x3 form's layout).
#include "bf16.h"
#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

constexpr int KA = SPARSE_KA;
constexpr int KM = SPARSE_KM;

__global__ __launch_bounds__(256) void sparse_rows_kernel(const double* __restrict__ A,
                                                          const int8_t* __restrict__ GM, int64_t n, int64_t np,
                                                          int64_t sM, const int* skip, SparseRows r) {
  const int b = blockIdx.y;
  if (skip && skip[b]) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;  // whole wave
  A += b * sM + i * np;
  GM += b * sM + i * np;
  int* colA = r.colA + ((int64_t)b * r.rows + i) * KA;
  double* valA = r.valA + ((int64_t)b * r.rows + i) * KA;
  int* colM = r.colM + ((int64_t)b * r.rows + i) * KM;
  const uint64_t below = (1ull << lane) - 1;
  int na = 0, nm = 0;
  // eight 64-column chunks per round, all loaded before the first is compacted (the
  // loads are unconditional: a column past n is read at a clamped in-row index and
  // ignored), so a wave keeps eight round trips in flight instead of one
  constexpr int U = 8;
  for (int64_t j0 = 0; j0 < n; j0 += 64 * U) {
    double av[U];
    int8_t gv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = min(j0 + 64 * u + lane, np - 1);
      av[u] = A[j];
      gv[u] = GM[j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + 64 * u + lane;
      const bool in = j < n;
      const double a = av[u];
      const bool ka = in && (a != 0.0), km = in && (gv[u] != 0) && (j <= i);
      const uint64_t ba = __ballot(ka), bm = __ballot(km);
      if (ka) {
        const int pos = na + __popcll(ba & below);
        if (pos < KA) {
          colA[pos] = (int)j;
          valA[pos] = a;
        }
      }
      if (km) {
        const int pos = nm + __popcll(bm & below);
        if (pos < KM) colM[pos] = (int)j;
      }
      na += __popcll(ba);
      nm += __popcll(bm);
    }
  }
  if (lane == 0) {
    int* cnt = r.cnt + ((int64_t)b * r.rows + i) * 2;
    cnt[0] = na;
    cnt[1] = nm;
  }
}

__global__ __launch_bounds__(256) void sparse_decide_kernel(int64_t n, const int* skip, SparseRows r, double* scal) {
  const int b = blockIdx.x;
  if (skip && skip[b]) {
    if (threadIdx.x == 0) {
      r.dense[b] = 1;
      r.dskip[b] = 1;
    }
    return;
  }
  const int* cnt = r.cnt + (int64_t)b * r.rows * 2;
  int over = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) over |= (cnt[2 * i] > KA) || (cnt[2 * i + 1] > KM);
  over = __syncthreads_or(over);
  if (threadIdx.x == 0) {
    r.dense[b] = over ? 1 : 0;
    r.dskip[b] = over ? 0 : 1;
    scal[(int64_t)b * SC_COUNT + SC_DENSE_PRODUCT] = over ? 1.0 : 0.0;
  }
}

// element (l, k) of Z: FP64, or hi + lo of the split layout (runs of 8 elements:
// 16 bytes of hi parts, then 16 bytes of lo parts)
template <bool SPLIT>
__device__ __forceinline__ double z_at(const void* Z, int64_t np, int l, int k) {
  if (SPLIT) {
    const uint8_t* run = static_cast<const uint8_t*>(Z) + ((int64_t)l * np + (k & ~7)) * 4 + (k & 7) * 2;
    const uint32_t hi = *reinterpret_cast<const uint16_t*>(run);
    const uint32_t lo = *reinterpret_cast<const uint16_t*>(run + 16);
    return (double)bf16_value(hi) + (double)bf16_value(lo);
  }
  return static_cast<const double*>(Z)[(int64_t)l * np + k];
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void sparse_product_kernel(const void* Z, int64_t sZ, int64_t n, int64_t np,
                                                             int64_t sM, const int* skip, SparseRows r,
                                                             double* __restrict__ P) {
  const int b = blockIdx.y;
  if ((skip && skip[b]) || r.dense[b]) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  Z = static_cast<const uint8_t*>(Z) + b * sZ;
  P += b * sM;
  const int64_t rb = (int64_t)b * r.rows;
  const int* colA = r.colA + rb * KA;
  const double* valA = r.valA + rb * KA;
  const int* cnt = r.cnt + rb * 2;
  const int ni = cnt[2 * i], nm = cnt[2 * i + 1];
  if (lane >= nm) return;
  const int j = r.colM[(rb + i) * KM + lane];
  const int nj = cnt[2 * (int64_t)j];
  // row i of A (the same for every lane) and row j (this lane's entry)
  int li[KA], kj[KA];
  double ai[KA], aj[KA];
#pragma unroll
  for (int q = 0; q < KA; ++q) {
    li[q] = q < ni ? colA[i * KA + q] : 0;
    ai[q] = q < ni ? valA[i * KA + q] : 0.0;
    kj[q] = q < nj ? colA[(int64_t)j * KA + q] : 0;
    aj[q] = q < nj ? valA[(int64_t)j * KA + q] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int p = 0; p < KA; ++p) {
    if (p < nj) {
      double x = 0.0;  // X_ik = (A Z)_ik, k = kj[p]
#pragma unroll
      for (int q = 0; q < KA; ++q)
        if (q < ni) x += ai[q] * z_at<SPLIT>(Z, np, li[q], kj[p]);
      acc += x * aj[p];
    }
  }
  P[i * np + j] = acc;
}

__global__ void mask_free_set_kernel(double* __restrict__ P, const int8_t* __restrict__ GM, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    if (GM[e] == 0) P[e] = 0.0;
}

}  // namespace

int mask_free_set(hipStream_t stream, double* P, const int8_t* GM, int64_t count) {
  if (count <= 0) return 0;
  const int blocks = (int)std::min<int64_t>((count + 255) / 256, 16384);
  hipLaunchKernelGGL(mask_free_set_kernel, dim3(blocks), dim3(256), 0, stream, P, GM, count);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int sparse_product(hipStream_t stream, const double* A, const int8_t* GM, const void* Z, int z_split, int64_t sZ,
                   int64_t n, int64_t np, int count, const int* skip, const SparseRows& r, double* scal, double* P) {
  if (count <= 0 || n <= 0) return 0;
  if (n > np || r.rows < np) return -1;
  const int64_t sM = np * np;
  const dim3 rows_grid((unsigned)((n + 3) / 4), count);
  hipLaunchKernelGGL(sparse_rows_kernel, rows_grid, dim3(256), 0, stream, A, GM, n, np, sM, skip, r);
  hipLaunchKernelGGL(sparse_decide_kernel, dim3(count), dim3(256), 0, stream, n, skip, r, scal);
  if (z_split)
    hipLaunchKernelGGL(sparse_product_kernel<true>, rows_grid, dim3(256), 0, stream, Z, sZ, n, np, sM, skip, r, P);
  else
    hipLaunchKernelGGL(sparse_product_kernel<false>, rows_grid, dim3(256), 0, stream, Z, sZ, n, np, sM, skip, r, P);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
