// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64), LDS-staged tiles.
//
//   C = alpha * op(A) * op(B) + beta * C      (row-major C, ldc)
//
// op(A) is M x K: TA = 0 reads A[m*lda + k], TA = 1 reads A[k*lda + m].
// op(B) is K x N: TB = 0 reads B[n*ldb + k], TB = 1 reads B[k*ldb + n].
// M, N are multiples of 128 and K of 16 (callers pad every matrix).
//
// Structure flags serve the blocked Cholesky / triangular-inverse / LAUUM code:
//   lower_out : compute only tiles on or below the tile diagonal (M == N);
//               diagonal tiles are written in full, callers read their lower part.
//   a_tri     : 1 = op(A) lower triangular (zero for k > m), 2 = upper (k < m);
//               the K range of a tile is clipped and the straddling slices masked.
//   b_tri     : 1 = op(B) lower triangular (zero for k < n), 2 = upper (k > n).
//   abort_flag: when non-null and abort_flag[z] is nonzero at launch, problem z
//               of the batch is skipped (a failed pivot earlier in the same
//               factorisation, or a problem that is not being iterated).
//
// Batching: grid.y walks a first batch dimension (strides sA, sB, sC) and grid.z
// a second one (strides zA, zB, zC), e.g. the groups of one problem and the
// problems of a batch.
//
// Workgroup: 256 threads = 4 wave64s in a 2x2 arrangement, 128x128 output tile,
// each wave owns 64x64 = 4x4 MFMA blocks (64 FP64 accumulators per lane).  BK=16
// slices of op(A) and op(B) are double-buffered in LDS ([row][k], k contiguous).
#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int LDK = BK + 2;  // 144-byte rows keep 16-byte alignment and spread banks

struct GemmF64Params {
  int M, N, K;
  int tiles_m, tiles_n;
  int lower_out, a_tri, b_tri;
  double alpha, beta;
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int64_t sA, sB, sC;  // grid.y batch strides (elements)
  int64_t zA, zB, zC;  // grid.z batch strides (elements)
  const int* abort_flag;
};

template <int TA>
__device__ __forceinline__ void load_a(const GemmF64Params& p, const double* A, int m0, int kt,
                                       int tid, double (&r)[8]) {
  if (TA == 0) {
    const int row = tid >> 1, kq = (tid & 1) * 8;
    const double2* src = reinterpret_cast<const double2*>(A + (int64_t)(m0 + row) * p.lda + kt + kq);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double2 v = src[i];
      r[2 * i] = v.x;
      r[2 * i + 1] = v.y;
    }
    if (p.a_tri) {
      const int m = m0 + row;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = kt + kq + i;
        if ((p.a_tri == 1 && k > m) || (p.a_tri == 2 && k < m)) r[i] = 0.0;
      }
    }
  } else {
    // one LDS row (= one m) per thread: coalesced 8-byte loads along m, 16-byte LDS stores
    const int mc = tid & 127, kh = (tid >> 7) * 8;
    const double* src = A + (int64_t)(kt + kh) * p.lda + m0 + mc;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = src[(int64_t)i * p.lda];
    if (p.a_tri) {
      const int m = m0 + mc;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = kt + kh + i;
        if ((p.a_tri == 1 && k > m) || (p.a_tri == 2 && k < m)) r[i] = 0.0;
      }
    }
  }
}

template <int TB>
__device__ __forceinline__ void load_b(const GemmF64Params& p, const double* B, int n0, int kt,
                                       int tid, double (&r)[8]) {
  if (TB == 0) {
    const int row = tid >> 1, kq = (tid & 1) * 8;
    const double2* src = reinterpret_cast<const double2*>(B + (int64_t)(n0 + row) * p.ldb + kt + kq);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double2 v = src[i];
      r[2 * i] = v.x;
      r[2 * i + 1] = v.y;
    }
    if (p.b_tri) {
      const int n = n0 + row;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = kt + kq + i;
        if ((p.b_tri == 1 && k < n) || (p.b_tri == 2 && k > n)) r[i] = 0.0;
      }
    }
  } else {
    const int nc = tid & 127, kh = (tid >> 7) * 8;
    const double* src = B + (int64_t)(kt + kh) * p.ldb + n0 + nc;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = src[(int64_t)i * p.ldb];
    if (p.b_tri) {
      const int n = n0 + nc;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = kt + kh + i;
        if ((p.b_tri == 1 && k < n) || (p.b_tri == 2 && k > n)) r[i] = 0.0;
      }
    }
  }
}

// store a register slice into LDS laid out [row][k]
template <int T>
__device__ __forceinline__ void store_slice(double (*S)[LDK], int tid, const double (&r)[8]) {
  if (T == 0) {
    const int row = tid >> 1, kq = (tid & 1) * 8;
    double2* dst = reinterpret_cast<double2*>(&S[row][kq]);
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[i] = make_double2(r[2 * i], r[2 * i + 1]);
  } else {
    const int mc = tid & 127, kh = (tid >> 7) * 8;
    double2* dst = reinterpret_cast<double2*>(&S[mc][kh]);
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[i] = make_double2(r[2 * i], r[2 * i + 1]);
  }
}

// ROLE only separates instantiations in profiles: 0 = factorisation/inverse
// updates, 1 = the preconditioned product A Z A.
template <int TA, int TB, int ROLE>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(GemmF64Params p) {
  if (p.abort_flag && p.abort_flag[blockIdx.z]) return;

  __shared__ __attribute__((aligned(16))) double As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) double Bs[2][BN][LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Contiguous tile ranges per XCD share operand panels in L2, but when the K
  // range depends on the tile (triangular operands) they would also give one XCD
  // all the long tiles; those launches keep the hardware's round-robin order.
  const int L = (p.a_tri || p.b_tri) ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  if (p.lower_out)
    lower_tile(L, p.tiles_m, ti, tj);
  else
    grouped_tile(L, p.tiles_m, p.tiles_n, ti, tj);
  const int m0 = ti * BM, n0 = tj * BN;

  const double* A = p.A + (int64_t)blockIdx.y * p.sA + (int64_t)blockIdx.z * p.zA;
  const double* B = p.B + (int64_t)blockIdx.y * p.sB + (int64_t)blockIdx.z * p.zB;
  double* C = p.C + (int64_t)blockIdx.y * p.sC + (int64_t)blockIdx.z * p.zC;

  int kbeg = 0, kend = p.K;
  if (p.a_tri == 1) kend = min(kend, m0 + BM);
  if (p.a_tri == 2) kbeg = max(kbeg, m0);
  if (p.b_tri == 1) kbeg = max(kbeg, n0);
  if (p.b_tri == 2) kend = min(kend, n0 + BN);

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  if (kbeg < kend) {
    double ra[8], rb[8];
    load_a<TA>(p, A, m0, kbeg, tid, ra);
    load_b<TB>(p, B, n0, kbeg, tid, rb);
    store_slice<TA>(As[0], tid, ra);
    store_slice<TB>(Bs[0], tid, rb);
    __syncthreads();
    int cur = 0;
    for (int kt = kbeg; kt < kend; kt += BK) {
      const bool more = kt + BK < kend;
      if (more) {
        load_a<TA>(p, A, m0, kt + BK, tid, ra);
        load_b<TB>(p, B, n0, kt + BK, tid, rb);
      }
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        double af[4], bf[4];
        const int kc = kk * 4 + (lane >> 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = As[cur][wm * 64 + i * 16 + (lane & 15)][kc];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][wn * 64 + j * 16 + (lane & 15)][kc];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
      if (more) {
        store_slice<TA>(As[cur ^ 1], tid, ra);
        store_slice<TB>(Bs[cur ^ 1], tid, rb);
      }
      __syncthreads();
      cur ^= 1;
    }
  }

  // D[r][c] of a 16x16 block sits in lane (c + 16*(r%4)), element r/4
  // (v_mfma_f64_16x16x4f64 output layout, checked on gfx950).
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + 4 * r + (lane >> 4);
        double* dst = C + (int64_t)row * p.ldc + col;
        double v = alpha * acc[i][j][r];
        if (beta != 0.0) v += beta * (*dst);
        *dst = v;
      }
    }
  }
}

}  // namespace

int gemm_f64(hipStream_t stream, int ta, int tb, int M, int N, int K, double alpha,
             const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
             int64_t ldc, int lower_out, int a_tri, int b_tri, const int* abort_flag, int batch,
             int64_t sA, int64_t sB, int64_t sC, int role, const ZBatch& zb) {
  if (M <= 0 || N <= 0 || batch <= 0 || zb.count <= 0) return 0;
  if (M % BM || N % BN || K % BK || K < 0) return -1;
  if (lower_out && M != N) return -1;
  GemmF64Params p;
  p.M = M;
  p.N = N;
  p.K = K;
  p.tiles_m = M / BM;
  p.tiles_n = N / BN;
  p.lower_out = lower_out;
  p.a_tri = a_tri;
  p.b_tri = b_tri;
  p.alpha = alpha;
  p.beta = beta;
  p.A = A;
  p.B = B;
  p.C = C;
  p.lda = lda;
  p.ldb = ldb;
  p.ldc = ldc;
  p.sA = sA;
  p.sB = sB;
  p.sC = sC;
  p.zA = zb.sA;
  p.zB = zb.sB;
  p.zC = zb.sC;
  p.abort_flag = abort_flag;
  const int tiles = lower_out ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  dim3 grid(tiles, batch, zb.count), block(256);
  if (role == 1 && ta == 0 && tb == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<0, 0, 1>), grid, block, 0, stream, p);
  else if (ta == 0 && tb == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<0, 0, 0>), grid, block, 0, stream, p);
  else if (ta == 0 && tb == 1)
    hipLaunchKernelGGL((gemm_f64_kernel<0, 1, 0>), grid, block, 0, stream, p);
  else if (ta == 1 && tb == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<1, 0, 0>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<1, 1, 0>), grid, block, 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
