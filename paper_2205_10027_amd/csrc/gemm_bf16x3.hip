// BF16x3 products for the preconditioned product A Z A (the BF16x3 mixed form).
//
// Each operand x is split into two bf16 parts: hi = x rounded to bf16 and
// lo = (x - hi) rounded to bf16, so x = hi + lo up to about 2^-17 |x|.  A product
// a b is formed as hi(a) hi(b) + hi(a) lo(b) + lo(a) hi(b) on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation; the dropped lo lo term is about
// 2^-18 |a b|.  The product only steers the step direction (eq. d_sol): the
// factor, log det, PD test, W and the KKT measure stay FP64.
//
// Split layout ("bf16x2"): row-major, 4 bytes per element.  Each run of 8
// consecutive elements of a row is stored as 16 bytes of hi parts followed by 16
// bytes of lo parts: exactly the 8 consecutive k that one lane feeds to one MFMA,
// so a fragment is one 16-byte LDS read.  The padded dimension is a multiple of
// 128, so a run never straddles two rows and the split of a matrix is a flat
// conversion of its element array.
//
// gemm_bf16x3_nt: C = A * B^T, A (M x K) and B (N x K) in split layout; 128x128
// output tile per workgroup, 4 wave64 of 64x64, 32 k per stage in double-buffered
// LDS (72 KB, two workgroups per CU).  C is written in split layout (the next
// product's operand) or as the FP64 lower triangle.
#include "bf16.h"
#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // (HIP's uint4 struct keeps arrays in scratch)

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int ROW = BK * 4 + 16;  // LDS bytes per tile row: 32 k x (hi, lo) x 2 B, + 16 B pad

struct GemmBf16Params {
  int M, N, K, tiles_m, tiles_n, lower_out;
  const uint8_t* A;  // split layout, row stride 4 * lda bytes
  const uint8_t* B;
  uint8_t* C;
  int64_t lda, ldb, ldc;  // elements
  int64_t zA, zB, zC;     // per-problem strides, elements
  const int* skip;        // per-problem skip flags (may be null)
};

// one 128-row x 32-k stage of a split operand: thread t copies 64 bytes of row t/2
__device__ __forceinline__ void load_stage(const uint8_t* P, int64_t ld, int r0, int kt, int tid, v4u (&r)[4]) {
  const v4u* src =
      reinterpret_cast<const v4u*>(P + (int64_t)(r0 + (tid >> 1)) * ld * 4 + (int64_t)kt * 4 + (tid & 1) * 64);
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = src[i];
}
__device__ __forceinline__ void store_stage(uint8_t* S, int tid, const v4u (&r)[4]) {
  v4u* dst = reinterpret_cast<v4u*>(S + (tid >> 1) * ROW + (tid & 1) * 64);
#pragma unroll
  for (int i = 0; i < 4; ++i) dst[i] = r[i];
}

template <int DOUBLE_OUT>
__global__ __launch_bounds__(256, 2) void gemm_bf16x3_nt_kernel(GemmBf16Params p) {
  if (p.skip && p.skip[blockIdx.z]) return;
  p.A += (int64_t)blockIdx.z * p.zA * 4;
  p.B += (int64_t)blockIdx.z * p.zB * 4;
  p.C += (int64_t)blockIdx.z * p.zC * (DOUBLE_OUT ? 8 : 4);
  __shared__ __attribute__((aligned(16))) uint8_t As[2][BM * ROW];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][BN * ROW];
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

  v4u ra[4], rb[4];
  load_stage(p.A, p.lda, m0, 0, tid, ra);
  load_stage(p.B, p.ldb, n0, 0, tid, rb);
  store_stage(As[0], tid, ra);
  store_stage(Bs[0], tid, rb);
  __syncthreads();
  // lane's fragment: row (lane & 15) of a 16-row block, k run (lane >> 4) of the stage
  const int frag = (lane & 15) * ROW + (lane >> 4) * 32;
  int cur = 0;
  for (int kt = 0; kt < p.K; kt += BK) {
    const bool more = kt + BK < p.K;
    if (more) {
      load_stage(p.A, p.lda, m0, kt + BK, tid, ra);
      load_stage(p.B, p.ldb, n0, kt + BK, tid, rb);
    }
    v8bf ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint8_t* a = As[cur] + (wm * 64 + i * 16) * ROW + frag;
      ah[i] = *reinterpret_cast<const v8bf*>(a);
      al[i] = *reinterpret_cast<const v8bf*>(a + 16);
      const uint8_t* b = Bs[cur] + (wn * 64 + i * 16) * ROW + frag;
      bh[i] = *reinterpret_cast<const v8bf*>(b);
      bl[i] = *reinterpret_cast<const v8bf*>(b + 16);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    if (more) {
      store_stage(As[cur ^ 1], tid, ra);
      store_stage(Bs[cur ^ 1], tid, rb);
    }
    __syncthreads();
    cur ^= 1;
  }
  // D[r][c] of a 16x16 block sits in lane (c + 16*(r/4)), element r%4
  // (v_mfma_f32_16x16x32_bf16 output layout, checked on gfx950).
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        const float x = acc[i][j][r];
        if (DOUBLE_OUT) {
          reinterpret_cast<double*>(p.C)[(int64_t)row * p.ldc + col] = (double)x;
        } else {
          const uint32_t h = bf16_bits(x);
          const uint32_t l = bf16_bits(x - bf16_value(h));
          uint16_t* dst = reinterpret_cast<uint16_t*>(p.C + (int64_t)row * p.ldc * 4 + (col >> 3) * 32 + (col & 7) * 2);
          dst[0] = (uint16_t)h;
          dst[8] = (uint16_t)l;
        }
      }
    }
}

// FP64 -> split layout; one run of 8 elements per thread and step (nothing when *skip)
__global__ void split_bf16x2_kernel(const double* __restrict__ src, uint8_t* __restrict__ dst, int64_t runs,
                                    const int* skip) {
  if (skip && *skip) return;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < runs; g += (int64_t)gridDim.x * blockDim.x) {
    const double2* s = reinterpret_cast<const double2*>(src + g * 8);
    uint32_t hi[4], lo[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = s[q];
      uint32_t h0, l0, h1, l1;
      split2(v.x, h0, l0);
      split2(v.y, h1, l1);
      hi[q] = h0 | (h1 << 16);
      lo[q] = l0 | (l1 << 16);
    }
    v4u* d = reinterpret_cast<v4u*>(dst + g * 32);
    d[0] = (v4u){hi[0], hi[1], hi[2], hi[3]};
    d[1] = (v4u){lo[0], lo[1], lo[2], lo[3]};
  }
}

}  // namespace

int gemm_bf16x3_nt(hipStream_t stream, int M, int N, int K, const void* A, int64_t lda, const void* B, int64_t ldb,
                   void* C, int64_t ldc, int c_is_double, int lower_out, const ZBatch& zb, const int* skip) {
  if (M <= 0 || N <= 0 || zb.count <= 0) return 0;
  if (M % BM || N % BN || K % BK || K <= 0) return -1;
  if (lower_out && (M != N || !c_is_double)) return -1;
  GemmBf16Params p;
  p.M = M;
  p.N = N;
  p.K = K;
  p.tiles_m = M / BM;
  p.tiles_n = N / BN;
  p.lower_out = lower_out;
  p.A = static_cast<const uint8_t*>(A);
  p.B = static_cast<const uint8_t*>(B);
  p.C = static_cast<uint8_t*>(C);
  p.lda = lda;
  p.ldb = ldb;
  p.ldc = ldc;
  p.zA = zb.sA;
  p.zB = zb.sB;
  p.zC = zb.sC;
  p.skip = skip;
  const int tiles = lower_out ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  if (c_is_double)
    hipLaunchKernelGGL(gemm_bf16x3_nt_kernel<1>, dim3(tiles, 1, zb.count), dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL(gemm_bf16x3_nt_kernel<0>, dim3(tiles, 1, zb.count), dim3(256), 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int split_bf16x2(hipStream_t stream, const double* src, void* dst, int64_t count, const int* skip) {
  if (count % 8) return -1;
  const int64_t runs = count / 8;
  const int blocks = (int)std::min<int64_t>((runs + 255) / 256, 16384);
  hipLaunchKernelGGL(split_bf16x2_kernel, dim3(blocks), dim3(256), 0, stream, src, static_cast<uint8_t*>(dst), runs,
                     skip);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
