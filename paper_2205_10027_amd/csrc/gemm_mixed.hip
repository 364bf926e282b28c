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
  const int L = xcd_remap(blockIdx.x, gridDim.x);
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

  const int kbeg = 0;
  float ra[16], rb[16];
  load_slice(p.A, p.lda, m0, kbeg, tid, ra);
  load_slice(p.B, p.ldb, n0, kbeg, tid, rb);
  store_slice(As[0], tid, ra);
  store_slice(Bs[0], tid, rb);
  __syncthreads();
  int cur = 0;
  for (int kt = 0; kt < p.K; kt += BK) {
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

__global__ void f64_to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t count) {
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; e < count;
       e += (int64_t)gridDim.x * blockDim.x * 2) {
    const double2 v = *reinterpret_cast<const double2*>(src + e);
    *reinterpret_cast<float2*>(dst + e) = make_float2((float)v.x, (float)v.y);
  }
}

}  // namespace

int gemm_f32_nt(hipStream_t stream, int M, int N, int K, const float* A, int64_t lda, const float* B, int64_t ldb,
                void* C, int64_t ldc, int c_is_double, int lower_out, const ZBatch& zb, const int* skip) {
  if (M <= 0 || N <= 0 || zb.count <= 0) return 0;
  if (M % BM || N % BN || K % BK || K <= 0) return -1;
  if (lower_out && M != N) return -1;
  GemmF32Params p;
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

int f64_to_f32(hipStream_t stream, const double* src, float* dst, int64_t count) {
  if (count % 2) return -1;
  const int blocks = (int)std::min<int64_t>((count / 2 + 255) / 256, 16384);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(blocks), dim3(256), 0, stream, src, dst, count);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
