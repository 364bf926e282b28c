// Reduced-precision GEMMs for the preconditioned product A Z A (the "mixed"
// forms): the product only steers the step direction (eq. d_sol), while the
// factor, log det, PD test, W and the KKT measure stay FP64.
//
// gemm_f32_nt: C = A * B^T with A (M x K), B (N x K) row-major FP32, FP32 MFMA
// (v_mfma_f32_16x16x4f32) with FP32 accumulation; C is written as float or as
// double.  Tiles: 128x128 output, 4 wave64 x 64x64, BK = 32 floats in
// double-buffered LDS; same XCD-aware order as the FP64 kernel.
#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int LDK = BK + 4;  // 144-byte rows: 16-byte aligned, banks spread

struct GemmF32Params {
  int M, N, K, tiles_m, tiles_n, lower_out;
  int k_from_row;  // with lower_out: k starts at the tile's first row (A = B upper-zero, e.g. V^T)
  const float* A;
  const float* B;
  void* C;
  int64_t lda, ldb, ldc;
  int64_t zA, zB, zC;  // grid.z (problem) strides, elements
  const int* skip;     // per-problem skip flags (may be null)
};

// one 128 x 32 float slice per operand: thread t loads row t/2, 16 floats
// (plain float registers: HIP's float4 struct keeps the prefetch in scratch)
__device__ __forceinline__ void load_slice(const float* P, int64_t ld, int r0, int kt, int tid, float (&r)[16]) {
  const float4* src = reinterpret_cast<const float4*>(P + (int64_t)(r0 + (tid >> 1)) * ld + kt + (tid & 1) * 16);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float4 v = src[i];
    r[4 * i] = v.x;
    r[4 * i + 1] = v.y;
    r[4 * i + 2] = v.z;
    r[4 * i + 3] = v.w;
  }
}
__device__ __forceinline__ void store_slice(float (*S)[LDK], int tid, const float (&r)[16]) {
  float4* dst = reinterpret_cast<float4*>(&S[tid >> 1][(tid & 1) * 16]);
#pragma unroll
  for (int i = 0; i < 4; ++i) dst[i] = make_float4(r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3]);
}

template <typename TC>
__global__ __launch_bounds__(256, 2) void gemm_f32_nt_kernel(GemmF32Params p) {
  if (p.skip && p.skip[blockIdx.z]) return;
  p.A += blockIdx.z * p.zA;
  p.B += blockIdx.z * p.zB;
  p.C = reinterpret_cast<char*>(p.C) + blockIdx.z * p.zC * (int64_t)sizeof(TC);
  __shared__ __attribute__((aligned(16))) float As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // with a K range that depends on the tile row, contiguous tile ranges per XCD
  // would give one XCD all the long tiles: keep the hardware's round-robin order
  // (lower_tile enumerates the long top bands first)
  const int L = p.k_from_row ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  if (p.lower_out)
    lower_tile(L, p.tiles_m, ti, tj);
  else
    grouped_tile(L, p.tiles_m, p.tiles_n, ti, tj);
  const int m0 = ti * BM, n0 = tj * BN;

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};

  const int kbeg = p.k_from_row ? m0 : 0;
  float ra[16], rb[16];
  load_slice(p.A, p.lda, m0, kbeg, tid, ra);
  load_slice(p.B, p.ldb, n0, kbeg, tid, rb);
  store_slice(As[0], tid, ra);
  store_slice(Bs[0], tid, rb);
  __syncthreads();
  int cur = 0;
  for (int kt = kbeg; kt < p.K; kt += BK) {
    const bool more = kt + BK < p.K;
    if (more) {
      load_slice(p.A, p.lda, m0, kt + BK, tid, ra);
      load_slice(p.B, p.ldb, n0, kt + BK, tid, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      float af[4], bf[4];
      const int kc = kk * 4 + (lane >> 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[cur][wm * 64 + i * 16 + (lane & 15)][kc];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][wn * 64 + j * 16 + (lane & 15)][kc];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      store_slice(As[cur ^ 1], tid, ra);
      store_slice(Bs[cur ^ 1], tid, rb);
    }
    __syncthreads();
    cur ^= 1;
  }
  // D[r][c] of a 16x16 block sits in lane (c + 16*(r/4)), element r%4
  // (v_mfma_f32_16x16x4f32 output layout, checked on gfx950).
  TC* C = reinterpret_cast<TC*>(p.C);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        C[(int64_t)row * p.ldc + col] = (TC)acc[i][j][r];
      }
    }
}

// ---- FP32 triangular inverse (the mixed-W iterations)
//
// T starts as L with its 128x128 diagonal blocks replaced by their inverses, zeros
// above the diagonal, in FP32; Tt = T^T.  Recursive doubling as in the FP64
// trtri_lower, each product as an NT GEMM on these two copies:
//   tmp^T = (T21 V11)^T   A = T21 (rows of T), B = rows of V11^T (rows of Tt),
//                         k >= the column tile (V11 lower), output transposed;
//   V21 = -V22 tmp        A = V22 (rows of T), B = rows of tmp^T,
//                         k < row tile + 128 (V22 lower), output written to T
//                         and, transposed, to Tt.
// At the end T = inv(L) and Tt = inv(L)^T.

struct TriF32Params {
  int M, N, K, tiles_m, tiles_n, kclip;  // kclip 1: k >= n0; 2: k < m0 + 128
  float alpha;
  const float* A;
  const float* B;
  float* C;   // may be null
  float* CT;  // transposed output, may be null
  int64_t lda, ldb, ldc, ldct;
  int64_t sA, sB, sC, sCT;  // grid.y (group) strides
  int64_t zA, zB, zC, zCT;  // grid.z (problem) strides
  const int* skip;
};

template <int KCLIP>
__global__ __launch_bounds__(256, 2) void gemm_f32_tri_kernel(TriF32Params p) {
  if (p.skip && p.skip[blockIdx.z]) return;
  const float* A = p.A + blockIdx.y * p.sA + blockIdx.z * p.zA;
  const float* B = p.B + blockIdx.y * p.sB + blockIdx.z * p.zB;
  __shared__ __attribute__((aligned(16))) float As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // longest K range first: kclip 1 shortens with the column tile, 2 lengthens with the row tile
  const int L = blockIdx.x;
  int ti, tj;
  if (KCLIP == 1) {
    tj = L / p.tiles_m;
    ti = L - tj * p.tiles_m;
  } else {
    const int q = L / p.tiles_n;
    tj = L - q * p.tiles_n;
    ti = p.tiles_m - 1 - q;
  }
  const int m0 = ti * BM, n0 = tj * BN;
  const int kbeg = (KCLIP == 1) ? n0 : 0;
  const int kend = (KCLIP == 2) ? min(p.K, m0 + BM) : p.K;

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  if (kbeg < kend) {
    float ra[16], rb[16];
    load_slice(A, p.lda, m0, kbeg, tid, ra);
    load_slice(B, p.ldb, n0, kbeg, tid, rb);
    store_slice(As[0], tid, ra);
    store_slice(Bs[0], tid, rb);
    __syncthreads();
    int cur = 0;
    for (int kt = kbeg; kt < kend; kt += BK) {
      const bool more = kt + BK < kend;
      if (more) {
        load_slice(A, p.lda, m0, kt + BK, tid, ra);
        load_slice(B, p.ldb, n0, kt + BK, tid, rb);
      }
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        float af[4], bf[4];
        const int kc = kk * 4 + (lane >> 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = As[cur][wm * 64 + i * 16 + (lane & 15)][kc];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][wn * 64 + j * 16 + (lane & 15)][kc];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
      if (more) {
        store_slice(As[cur ^ 1], tid, ra);
        store_slice(Bs[cur ^ 1], tid, rb);
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  float* C = p.C ? p.C + blockIdx.y * p.sC + blockIdx.z * p.zC : nullptr;
  float* CT = p.CT ? p.CT + blockIdx.y * p.sCT + blockIdx.z * p.zCT : nullptr;
  // D[r][c] of a 16x16 block sits in lane (c + 16*(r/4)), element r%4
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
      const int row0 = m0 + wm * 64 + i * 16 + 4 * (lane >> 4);
      const v4f v = acc[i][j] * p.alpha;
      if (C) {
#pragma unroll
        for (int r = 0; r < 4; ++r) C[(int64_t)(row0 + r) * p.ldc + col] = v[r];
      }
      if (CT) *reinterpret_cast<v4f*>(CT + (int64_t)col * p.ldct + row0) = v;
    }
}

// T, Tt (FP32, np x np) from the factor L (lower) and its diagonal-block inverses
// Dinv (np x 128, ld 128); 64x64 tiles through LDS so T and Tt are both written
// along rows.
__global__ __launch_bounds__(256) void tri_init_f32_kernel(const double* __restrict__ L, const double* __restrict__ Dinv,
                                                           int64_t np, float* __restrict__ T, float* __restrict__ Tt,
                                                           int64_t sL, int64_t sD, int64_t sT, const int* skip) {
  if (skip && skip[blockIdx.z]) return;
  L += blockIdx.z * sL;
  Dinv += blockIdx.z * sD;
  T += blockIdx.z * sT;
  Tt += blockIdx.z * sT;
  __shared__ float t[64][65];
  const int bi = blockIdx.x, bj = blockIdx.y;  // tile rows i, columns j of T
  const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)bi * 64, j0 = (int64_t)bj * 64;
  if (bj > bi) {  // above the diagonal: zeros in T, and in Tt below it
    for (int r = r0; r < 64; r += 4) {
      T[(i0 + r) * np + j0 + c] = 0.f;
      Tt[(j0 + r) * np + i0 + c] = 0.f;
    }
    return;
  }
  const bool same_block = (bi >> 1) == (bj >> 1);  // inside one 128x128 diagonal block
  for (int r = r0; r < 64; r += 4) {
    const int64_t i = i0 + r, j = j0 + c;
    float v = 0.f;
    if (j <= i)
      v = same_block ? (float)Dinv[(i >> 7) * 128 * 128 + (i & 127) * 128 + (j & 127)] : (float)L[i * np + j];
    T[i * np + j] = v;
    t[r][c] = v;
  }
  __syncthreads();
  for (int r = r0; r < 64; r += 4) Tt[(j0 + r) * np + i0 + c] = t[c][r];
}

__global__ void f64_to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t count) {
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; e < count;
       e += (int64_t)gridDim.x * blockDim.x * 2) {
    const double2 v = *reinterpret_cast<const double2*>(src + e);
    *reinterpret_cast<float2*>(dst + e) = make_float2((float)v.x, (float)v.y);
  }
}

}  // namespace

int gemm_f32_nt(hipStream_t stream, int M, int N, int K, const float* A, int64_t lda, const float* B, int64_t ldb,
                void* C, int64_t ldc, int c_is_double, int lower_out, const ZBatch& zb, const int* skip,
                int k_from_row) {
  if (M <= 0 || N <= 0 || zb.count <= 0) return 0;
  if (M % BM || N % BN || K % BK || K <= 0) return -1;
  if (lower_out && M != N) return -1;
  if (k_from_row && !lower_out) return -1;
  GemmF32Params p;
  p.k_from_row = k_from_row;
  p.M = M;
  p.N = N;
  p.K = K;
  p.tiles_m = M / BM;
  p.tiles_n = N / BN;
  p.lower_out = lower_out;
  p.A = A;
  p.B = B;
  p.C = C;
  p.lda = lda;
  p.ldb = ldb;
  p.ldc = ldc;
  p.zA = zb.sA;
  p.zB = zb.sB;
  p.zC = zb.sC;
  p.skip = skip;
  const int tiles = lower_out ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  if (c_is_double)
    hipLaunchKernelGGL(gemm_f32_nt_kernel<double>, dim3(tiles, 1, zb.count), dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL(gemm_f32_nt_kernel<float>, dim3(tiles, 1, zb.count), dim3(256), 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

namespace {
int launch_tri(hipStream_t stream, int kclip, int M, int N, int K, float alpha, const float* A, int64_t lda,
               const float* B, int64_t ldb, float* C, int64_t ldc, float* CT, int64_t ldct, int groups, int64_t sA,
               int64_t sB, int64_t sC, int64_t sCT, int count, int64_t zA, int64_t zB, int64_t zC, int64_t zCT,
               const int* skip) {
  if (M % BM || N % BN || K % BK) return -1;
  TriF32Params p;
  p.M = M;
  p.N = N;
  p.K = K;
  p.tiles_m = M / BM;
  p.tiles_n = N / BN;
  p.kclip = kclip;
  p.alpha = alpha;
  p.A = A;
  p.B = B;
  p.C = C;
  p.CT = CT;
  p.lda = lda;
  p.ldb = ldb;
  p.ldc = ldc;
  p.ldct = ldct;
  p.sA = sA;
  p.sB = sB;
  p.sC = sC;
  p.sCT = sCT;
  p.zA = zA;
  p.zB = zB;
  p.zC = zC;
  p.zCT = zCT;
  p.skip = skip;
  const dim3 grid(p.tiles_m * p.tiles_n, groups, count);
  if (kclip == 1)
    hipLaunchKernelGGL(gemm_f32_tri_kernel<1>, grid, dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL(gemm_f32_tri_kernel<2>, grid, dim3(256), 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
}  // namespace

int trtri_f32(hipStream_t stream, const double* L, const double* Dinv, int64_t np, float* T, float* Tt, float* tmp,
              int count, int64_t sL, int64_t sD, int64_t sT, int64_t sTmp, const int* skip) {
  if (np % 128 || count <= 0) return np % 128 ? -1 : 0;
  const int T64 = (int)(np / 64);
  hipLaunchKernelGGL(tri_init_f32_kernel, dim3(T64, T64, count), dim3(256), 0, stream, L, Dinv, np, T, Tt, sL, sD,
                     sT, skip);
  if (hipGetLastError() != hipSuccess) return -2;
  const int64_t n = np;
  for (int64_t s = 128; s < n; s *= 2) {
    const int64_t gs = 2 * s * (np + 1);  // group stride inside T and Tt
    const int full = (int)(n / (2 * s));
    int rc;
    if (full > 0) {
      // tmp^T = (T21 V11)^T, one s x s tmp^T per group
      rc = launch_tri(stream, 1, (int)s, (int)s, (int)s, 1.f, T + s * np, np, Tt, np, nullptr, 0, tmp, s, full,
                      gs, gs, 0, s * s, count, sT, sT, 0, sTmp, skip);
      if (rc) return rc;
      // V21 = -V22 tmp into T21 and, transposed, into Tt
      rc = launch_tri(stream, 2, (int)s, (int)s, (int)s, -1.f, T + s * (np + 1), np, tmp, s, T + s * np, np,
                      Tt + s, np, full, gs, s * s, gs, gs, count, sT, sTmp, sT, sT, skip);
      if (rc) return rc;
    }
    const int64_t base = (int64_t)full * 2 * s;
    const int64_t n2 = n - base - s;
    if (n2 > 0) {
      rc = launch_tri(stream, 1, (int)n2, (int)s, (int)s, 1.f, T + (base + s) * np + base, np, Tt + base * np + base,
                      np, nullptr, 0, tmp, n2, 1, 0, 0, 0, 0, count, sT, sT, 0, sTmp, skip);
      if (rc) return rc;
      rc = launch_tri(stream, 2, (int)n2, (int)s, (int)n2, -1.f, T + (base + s) * (np + 1), np, tmp, n2,
                      T + (base + s) * np + base, np, Tt + base * np + base + s, np, 1, 0, 0, 0, 0, count, sT,
                      sTmp, sT, sT, skip);
      if (rc) return rc;
    }
  }
  return 0;
}

int f64_to_f32(hipStream_t stream, const double* src, float* dst, int64_t count) {
  if (count % 2) return -1;
  const int blocks = (int)std::min<int64_t>((count / 2 + 255) / 256, 16384);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(blocks), dim3(256), 0, stream, src, dst, count);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
