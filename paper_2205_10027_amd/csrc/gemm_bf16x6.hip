// FP32-accurate products on the BF16 matrix cores for W = A^-1 = V^T V,
// V = inv(L), in the mixed-W iterations (BF16x6).
//
// An FP32 value x is split into three bf16 parts, x1 = x rounded to bf16,
// x2 = (x - x1) rounded, x3 = x - x1 - x2 (exact: 24 significant bits in three
// 8-bit parts, barring underflow).  A product x y is formed from the six partial
// products x1 y1, x1 y2, x2 y1, x1 y3, x2 y2, x3 y1 on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation; each partial product is exact in FP32 and the three dropped
// ones (x2 y3, x3 y2, x3 y3) are below 2.1 * 2^-24 |x y| together, so the result has
// the accuracy of an FP32 product at six BF16 MFMA passes instead of one FP32 pass
// (16x fewer MFMA cycles per flop on gfx950).
//
// Split layout ("bf16x3"): row-major, 6 bytes per element.  Each run of 8
// consecutive elements of a row is stored as 16 bytes of x1 parts, 16 of x2, 16 of
// x3: the 8 consecutive k one lane feeds to one MFMA, so each fragment is one
// 16-byte LDS read.  Rows are multiples of 128 elements, so a 32-k stage of a row
// is 192 contiguous bytes.
//
// gemm_bf16x6_nt: C = tril(A B^T) in FP64, A and B (M x K, N x K) split; 128x128
// output tiles on and below the diagonal, 4 wave64 of 64x64, 32 k per stage through
// one LDS buffer (53 KB, two workgroups per CU) with the next stage prefetched in
// registers.  k_from_row starts each tile's K range at its first row (A[m][k] = 0
// for k < m, as for A = V^T with V lower triangular); tiles then run in launch
// order, longest K range first.
#include "bf16.h"
#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int T6 = 128, BK6 = 32;
constexpr int RUN6 = 48;                    // bytes per run of 8 elements
constexpr int STAGE6 = BK6 / 8 * RUN6;      // 192 bytes of a row per stage
constexpr int ROW6 = STAGE6 + 16;           // LDS row stride (16-byte pad)

struct GemmBf6Params {
  int K, tiles_m, k_from_row;
  const uint8_t* A;  // split layout, row stride 6 * lda bytes
  const uint8_t* B;
  double* C;
  int64_t lda, ldb, ldc;  // elements
  int64_t zA, zB, zC;     // per-problem strides: bytes for A and B, elements for C
  const int* skip;
};

// thread t stages 96 bytes (two runs) of row t/2 of a 128-row operand slice
__device__ __forceinline__ void load6(const uint8_t* P, int64_t ld, int r0, int kt, int tid, v4u (&r)[6]) {
  const v4u* src = reinterpret_cast<const v4u*>(P + (int64_t)(r0 + (tid >> 1)) * ld * 6 + (int64_t)kt * 6 +
                                                (tid & 1) * (STAGE6 / 2));
#pragma unroll
  for (int i = 0; i < 6; ++i) r[i] = src[i];
}
__device__ __forceinline__ void store6(uint8_t* S, int tid, const v4u (&r)[6]) {
  v4u* dst = reinterpret_cast<v4u*>(S + (tid >> 1) * ROW6 + (tid & 1) * (STAGE6 / 2));
#pragma unroll
  for (int i = 0; i < 6; ++i) dst[i] = r[i];
}

// acc += A[m0.., kbeg..kend) B[n0.., kbeg..kend)^T for the 4 wave64 of a 128x128
// tile (wave (wm, wn) owns rows wm*64.., columns wn*64..): 32-k stages through one
// LDS buffer per operand, the next stage prefetched in registers.  kmask (when
// `masked`): the 128-wide K chunks to multiply (bit c: k in [128c, 128c + 128));
// the others contribute exact zeros and are not read.
__device__ __forceinline__ void tile_product(const uint8_t* A, int64_t lda, const uint8_t* B, int64_t ldb, int m0,
                                             int n0, int kbeg, int kend, uint8_t* As, uint8_t* Bs, v4f (&acc)[4][4],
                                             int tid, bool masked = false, uint64_t kmask = ~0ull) {
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  if (masked) {
    if (!kmask) return;
    kbeg = max(kbeg, (int)(__builtin_ctzll(kmask) << 7));
  }
  if (kbeg >= kend) return;
  // the stage after kt: the next one, or with a mask the first of the next chunk in it
  auto next_k = [&](int kt) -> int {
    const int nk = kt + BK6;
    if (!masked || (nk & 127)) return nk;
    const int c = kt >> 7;
    const uint64_t later = (c >= 63) ? 0ull : (kmask & (~0ull << (c + 1)));
    return later ? (int)(__builtin_ctzll(later) << 7) : kend;
  };
  v4u ra[6], rb[6];
  load6(A, lda, m0, kbeg, tid, ra);
  load6(B, ldb, n0, kbeg, tid, rb);
  // lane's fragment: row (lane & 15) of a 16-row block, run (lane >> 4) of the stage
  const int frag = (lane & 15) * ROW6 + (lane >> 4) * RUN6;
  for (int kt = kbeg; kt < kend;) {
    store6(As, tid, ra);
    store6(Bs, tid, rb);
    __syncthreads();
    const int nk = next_k(kt);
    if (nk < kend) {
      load6(A, lda, m0, nk, tid, ra);
      load6(B, ldb, n0, nk, tid, rb);
    }
    v8bf a1[4], a2[4], a3[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint8_t* s = As + (wm * 64 + i * 16) * ROW6 + frag;
      a1[i] = *reinterpret_cast<const v8bf*>(s);
      a2[i] = *reinterpret_cast<const v8bf*>(s + 16);
      a3[i] = *reinterpret_cast<const v8bf*>(s + 32);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint8_t* s = Bs + (wn * 64 + j * 16) * ROW6 + frag;
      const v8bf b1 = *reinterpret_cast<const v8bf*>(s);
      const v8bf b2 = *reinterpret_cast<const v8bf*>(s + 16);
      const v8bf b3 = *reinterpret_cast<const v8bf*>(s + 32);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v4f c = acc[i][j];
        // smallest terms first
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[i], b1, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[i], b2, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[i], b3, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[i], b1, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[i], b2, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[i], b1, c, 0, 0, 0);
        acc[i][j] = c;
      }
    }
    __syncthreads();
    kt = nk;
  }
}

__global__ __launch_bounds__(256, 2) void gemm_bf16x6_nt_kernel(GemmBf6Params p) {
  if (p.skip && p.skip[blockIdx.z]) return;
  p.A += (int64_t)blockIdx.z * p.zA;
  p.B += (int64_t)blockIdx.z * p.zB;
  p.C += (int64_t)blockIdx.z * p.zC;
  __shared__ __attribute__((aligned(16))) uint8_t As[T6 * ROW6];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[T6 * ROW6];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // clipped K ranges differ per tile: keep the hardware's round-robin over XCDs,
  // lower_tile enumerates the long top bands first
  const int L = p.k_from_row ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  lower_tile(L, p.tiles_m, ti, tj);
  const int m0 = ti * T6, n0 = tj * T6;

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  tile_product(p.A, p.lda, p.B, p.ldb, m0, n0, p.k_from_row ? m0 : 0, p.K, As, Bs, acc, tid);
  // D[r][c] of a 16x16 block sits in lane (c + 16*(r/4)), element r%4
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        p.C[(int64_t)row * p.ldc + col] = (double)acc[i][j][r];
      }
    }
}

// ---- the three-part split of single FP32 values, and stores of them
__device__ __forceinline__ void split3(float x, uint32_t& h1, uint32_t& h2, uint32_t& h3) {
  h1 = bf16_bits(x);
  const float r1 = x - bf16_value(h1);  // exact
  h2 = bf16_bits(r1);
  h3 = bf16_bits(r1 - bf16_value(h2));  // exact
}
// a run of 8 consecutive elements (row, col0 .. col0 + 7), col0 a multiple of 8:
// three 16-byte stores
__device__ __forceinline__ void store_run(uint8_t* M, int64_t ld, int64_t row, int64_t col0, const float (&x)[8]) {
  uint32_t p1[4], p2[4], p3[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t a1, a2, a3, b1, b2, b3;
    split3(x[2 * q], a1, a2, a3);
    split3(x[2 * q + 1], b1, b2, b3);
    p1[q] = a1 | (b1 << 16);
    p2[q] = a2 | (b2 << 16);
    p3[q] = a3 | (b3 << 16);
  }
  v4u* d = reinterpret_cast<v4u*>(M + (row * ld + col0) * 6);
  d[0] = (v4u){p1[0], p1[1], p1[2], p1[3]};
  d[1] = (v4u){p2[0], p2[1], p2[2], p2[3]};
  d[2] = (v4u){p3[0], p3[1], p3[2], p3[3]};
}

// ---- triangular inverse on the split copies (the mixed-W iterations)
//
// T starts as L with its 128x128 diagonal blocks replaced by their inverses, zeros
// above the diagonal, rounded to FP32 and split; Tt = T^T.  Recursive doubling, each
// product an NT GEMM on the split copies:
//   tmp^T = (T21 V11)^T   A = T21 (rows of T), B = rows of V11^T (rows of Tt),
//                         k >= the column tile (V11 lower), output transposed;
//   V21 = -V22 tmp        A = V22 (rows of T), B = rows of tmp^T,
//                         k < row tile + 128 (V22 lower), output written to T
//                         and, transposed, to Tt.
// Every output is rounded to FP32 and split again.  At the end T = inv(L) and
// Tt = inv(L)^T, split.
struct TriBf6Params {
  int M, N, K, tiles_m, tiles_n;
  float alpha;
  const uint8_t* A;
  const uint8_t* B;
  uint8_t* C;   // may be null
  uint8_t* CT;  // transposed output, may be null
  int64_t lda, ldb, ldc, ldct;  // elements
  int64_t sA, sB, sC, sCT;      // grid.y (group) strides, bytes
  int64_t zA, zB, zC, zCT;      // grid.z (problem) strides, bytes
  const int* skip;
  // optional zero-block map of the factor L (ZBatch::nz layout): T21 of group g is L's
  // rows nz_row0 + g nz_gstep.. and columns nz_col0 + g nz_gstep .. + nz_w, untouched
  // by the earlier levels.  KCLIP 1 (A = T21): a tile whose T21 rows are zero in every
  // panel of its K range is zero.  KCLIP 2 (B = tmp^T, tmp = T21 V11): tmp's rows are
  // zero where T21's are, so K stops after tmp's last nonzero 64-row block.
  const uint8_t* nz;
  int64_t snz;
  int nz_chunks, nz_row0, nz_col0, nz_gstep, nz_w;
};

// rows of the output tile staged as FP32 in LDS for whole-run stores (64 rows at a time)
constexpr int STG_LD = T6 + 4;
static_assert(64 * STG_LD * 4 <= 2 * T6 * ROW6, "staging fits in the operand buffers");

template <int KCLIP>
__global__ __launch_bounds__(256, 2) void gemm_bf16x6_tri_kernel(TriBf6Params p) {
  if (p.skip && p.skip[blockIdx.z]) return;
  const uint8_t* A = p.A + blockIdx.y * p.sA + blockIdx.z * p.zA;
  const uint8_t* B = p.B + blockIdx.y * p.sB + blockIdx.z * p.zB;
  __shared__ __attribute__((aligned(16))) uint8_t lds[2 * T6 * ROW6];
  uint8_t* const As = lds;
  uint8_t* const Bs = lds + T6 * ROW6;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // longest K range first: KCLIP 1 shortens with the column tile, 2 lengthens with the row tile
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
  const int m0 = ti * T6, n0 = tj * T6;
  const int kbeg = (KCLIP == 1) ? n0 : 0;
  int kend = (KCLIP == 2) ? min(p.K, m0 + T6) : p.K;
  bool masked = false;
  uint64_t kmask = ~0ull;
  if (p.nz) {
    const uint8_t* f = p.nz + (int64_t)blockIdx.z * p.snz;
    const int r0 = p.nz_row0 + (int)blockIdx.y * p.nz_gstep;  // global row of T21's row 0
    const int c0 = p.nz_col0 + (int)blockIdx.y * p.nz_gstep;  // global column of T21's column 0
    if (KCLIP == 1 && (p.K >> 7) <= 64) {
      // K chunk c (128 columns of T21, panel (c0 >> 7) + c of L) is multiplied only
      // if the tile's 128 rows of T21 have a nonzero block in it: lane c of wave 0
      // looks it up
      __shared__ unsigned long long kmask_sh;
      if (wave == 0) {
        int on = 0;
        if (lane < (p.K >> 7) && 128 * lane + 128 > kbeg && 128 * lane < kend) {
          const uint8_t* fs = f + (int64_t)((c0 >> 7) + lane) * p.nz_chunks + ((r0 + m0) >> 6);
          on = fs[0] | fs[1];
        }
        const unsigned long long bal = __ballot(on);
        if (lane == 0) kmask_sh = bal;
      }
      __syncthreads();
      kmask = kmask_sh;
      masked = true;
    } else if (KCLIP == 1) {
      // every thread reads its share of the (panel, 64-row block) entries, all loads
      // independent, then one workgroup-wide reduction
      const int q0 = (c0 + kbeg) >> 7, nq = ((c0 + kend - 1) >> 7) - q0 + 1;
      int any = 0;
      for (int e = tid; e < 2 * nq; e += 256)
        any |= f[(int64_t)(q0 + (e >> 1)) * p.nz_chunks + ((r0 + m0) >> 6) + (e & 1)];
      if (!__syncthreads_or(any)) kend = kbeg;
    } else if ((p.K >> 7) <= 64) {
      // tmp's row chunk c (128 rows: tmp = T21 V11) is nonzero only where T21's rows
      // are: bit c of the mask when any panel of T21 has a nonzero block in them
      __shared__ unsigned long long kmask2_sh;
      if (tid == 0) kmask2_sh = 0ull;
      __syncthreads();
      const int q0 = c0 >> 7, nq = p.nz_w >> 7, nch = p.K >> 6;
      unsigned long long mine = 0ull;
      for (int e = tid; e < nch * nq; e += 256) {
        const int c = e / nq, q = q0 + e - (e / nq) * nq;
        if (f[(int64_t)q * p.nz_chunks + (r0 >> 6) + c]) mine |= 1ull << (c >> 1);
      }
      if (mine) atomicOr(&kmask2_sh, mine);
      __syncthreads();
      kmask = kmask2_sh;
      masked = true;
    } else {
      __shared__ int last[4];
      const int q0 = c0 >> 7, nq = p.nz_w >> 7, nch = p.K >> 6;
      int mine = -1;
      for (int e = tid; e < nch * nq; e += 256) {
        const int c = e / nq, q = q0 + e - (e / nq) * nq;
        if (f[(int64_t)q * p.nz_chunks + (r0 >> 6) + c]) mine = max(mine, c);
      }
      for (int off = 32; off > 0; off >>= 1) mine = max(mine, __shfl_xor(mine, off));
      if (lane == 0) last[wave] = mine;
      __syncthreads();
      const int cmax = max(max(last[0], last[1]), max(last[2], last[3]));
      kend = min(kend, 64 * (cmax + 1));
    }
  }

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  tile_product(A, p.lda, B, p.ldb, m0, n0, kbeg, kend, As, Bs, acc, tid, masked, kmask);
  uint8_t* C = p.C ? p.C + blockIdx.y * p.sC + blockIdx.z * p.zC : nullptr;
  uint8_t* CT = p.CT ? p.CT + blockIdx.y * p.sCT + blockIdx.z * p.zCT : nullptr;
  // The tile leaves through LDS in two halves of 64 rows (tile_product ends with a
  // barrier, so the operand buffers are free): every store is a whole run of 8
  // consecutive elements (three 16-byte stores), of C's rows and of CT's rows.
  // D[r][c] of a 16x16 block sits in lane (c + 16*(r/4)), element r%4.
  float(*st)[STG_LD] = reinterpret_cast<float(*)[STG_LD]>(lds);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (wm == h) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const v4f v = acc[i][j] * p.alpha;
#pragma unroll
          for (int r = 0; r < 4; ++r) st[i * 16 + 4 * (lane >> 4) + r][wn * 64 + j * 16 + (lane & 15)] = v[r];
        }
    }
    __syncthreads();
    if (C) {
      // 64 rows x 16 runs
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int g = tid + 256 * q, r = g >> 4, run = g & 15;
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = st[r][8 * run + e];
        store_run(C, p.ldc, m0 + 64 * h + r, n0 + 8 * run, x);
      }
    }
    if (CT) {
      // 128 rows of CT (the tile's columns) x 8 runs of this half's 64 rows
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int g = tid + 256 * q, col = g & 127, run = g >> 7;
        float y[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) y[e] = st[8 * run + e][col];
        store_run(CT, p.ldct, n0 + col, m0 + 64 * h + 8 * run, y);
      }
    }
    __syncthreads();
  }
}

// T and Tt (split) from the factor L (lower, FP64) and its diagonal-block inverses
// Dinv (np x 128, ld 128): a 64x64 tile of T goes through LDS, then every thread
// writes whole runs of T's rows and of Tt's rows.
// With the factor's zero-block map (nz, every first doubling product masked by it):
// a tile below the diagonal blocks is read only as T21 of its level, and only when
// its 128-row block has a nonzero block in its panel; tri<2> overwrites it (and its
// transpose in Tt) before anything else reads it.  So only those tiles of T, and
// the diagonal blocks of both copies, are written.
__global__ __launch_bounds__(256) void tri_init_bf16x6_kernel(const double* __restrict__ L,
                                                             const double* __restrict__ Dinv, int64_t np,
                                                             uint8_t* __restrict__ T, uint8_t* __restrict__ Tt,
                                                             int64_t sL, int64_t sD, int64_t sT, int64_t sTt,
                                                             const int* skip, const uint8_t* nz, int64_t snz,
                                                             int nz_chunks) {
  if (skip && skip[blockIdx.z]) return;
  const int bi = blockIdx.x, bj = blockIdx.y;  // tile rows i, columns j of T
  // Tiles of T above the 128x128 diagonal blocks (and their transposes in Tt) are
  // zero and never read: every later product clips its K range at 128-tile
  // granularity to the triangle (the doubling products, V^T V), so only the zeros
  // inside the diagonal blocks are read.  They are not written.
  if ((bj >> 1) > (bi >> 1)) return;
  const bool off_block = (bj >> 1) < (bi >> 1);
  if (nz && off_block) {
    const uint8_t* f = nz + (int64_t)blockIdx.z * snz + (int64_t)(bj >> 1) * nz_chunks;
    if (!(f[bi & ~1] | f[bi | 1])) return;
  }
  const bool write_tt = !(nz && off_block);
  L += blockIdx.z * sL;
  Dinv += blockIdx.z * sD;
  T += blockIdx.z * sT;
  Tt += blockIdx.z * sTt;
  __shared__ float t[64][65];
  const int tid = threadIdx.x, c = tid & 63, r0 = tid >> 6;
  const int64_t i0 = (int64_t)bi * 64, j0 = (int64_t)bj * 64;
  const bool same_block = (bi >> 1) == (bj >> 1);  // inside one 128x128 diagonal block
  for (int r = r0; r < 64; r += 4) {
    const int64_t i = i0 + r, j = j0 + c;
    float v = 0.f;
    if (bj <= bi && j <= i)
      v = same_block ? (float)Dinv[(i >> 7) * 128 * 128 + (i & 127) * 128 + (j & 127)] : (float)L[i * np + j];
    t[r][c] = v;
  }
  __syncthreads();
  // 64 rows x 8 runs of T's tile and of Tt's tile (its transpose), two of each per thread
  for (int g = tid; g < 512; g += 256) {
    const int r = g >> 3, q = g & 7;
    float x[8], y[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      x[e] = t[r][8 * q + e];
      y[e] = t[8 * q + e][r];
    }
    store_run(T, np, i0 + r, j0 + 8 * q, x);
    if (write_tt) store_run(Tt, np, j0 + r, i0 + 8 * q, y);
  }
}

}  // namespace

int gemm_bf16x6_lower(hipStream_t stream, int N, int K, const void* A, int64_t lda, const void* B, int64_t ldb,
                      double* C, int64_t ldc, int k_from_row, int count, int64_t zA_bytes, int64_t zB_bytes,
                      int64_t zC, const int* skip) {
  if (N <= 0 || count <= 0) return 0;
  if (N % T6 || K % BK6 || K <= 0) return -1;
  GemmBf6Params p;
  p.K = K;
  p.tiles_m = N / T6;
  p.k_from_row = k_from_row;
  p.A = static_cast<const uint8_t*>(A);
  p.B = static_cast<const uint8_t*>(B);
  p.C = C;
  p.lda = lda;
  p.ldb = ldb;
  p.ldc = ldc;
  p.zA = zA_bytes;
  p.zB = zB_bytes;
  p.zC = zC;
  p.skip = skip;
  const int tiles = p.tiles_m * (p.tiles_m + 1) / 2;
  hipLaunchKernelGGL(gemm_bf16x6_nt_kernel, dim3(tiles, 1, count), dim3(256), 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

namespace {
struct TriZeros {
  const uint8_t* nz = nullptr;
  int64_t snz = 0;
  int chunks = 0;
};
int launch_tri6(hipStream_t stream, int kclip, int M, int N, int K, float alpha, const uint8_t* A, int64_t lda,
                const uint8_t* B, int64_t ldb, uint8_t* C, int64_t ldc, uint8_t* CT, int64_t ldct, int groups,
                int64_t sA, int64_t sB, int64_t sC, int64_t sCT, int count, int64_t zA, int64_t zB, int64_t zC,
                int64_t zCT, const int* skip, const TriZeros& zr = TriZeros(), int row0 = 0, int col0 = 0,
                int gstep = 0, int width = 0) {
  if (M % T6 || N % T6 || K % BK6) return -1;
  TriBf6Params p;
  p.nz = zr.nz;
  p.snz = zr.snz;
  p.nz_chunks = zr.chunks;
  p.nz_row0 = row0;
  p.nz_col0 = col0;
  p.nz_gstep = gstep;
  p.nz_w = width;
  p.M = M;
  p.N = N;
  p.K = K;
  p.tiles_m = M / T6;
  p.tiles_n = N / T6;
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
    hipLaunchKernelGGL(gemm_bf16x6_tri_kernel<1>, grid, dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL(gemm_bf16x6_tri_kernel<2>, grid, dim3(256), 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
}  // namespace

int trtri_bf16x6(hipStream_t stream, const double* L, const double* Dinv, int64_t np, void* Tv, void* Ttv, void* tmpv,
                 int count, int64_t sL, int64_t sD, int64_t sT, int64_t sTt, int64_t sTmp, const int* skip,
                 const uint8_t* nz, int64_t snz) {
  if (np % 128 || count <= 0) return np % 128 ? -1 : 0;
  TriZeros zr;
  zr.nz = nz;
  zr.snz = snz;
  zr.chunks = (int)(np / 64);
  uint8_t* T = static_cast<uint8_t*>(Tv);
  uint8_t* Tt = static_cast<uint8_t*>(Ttv);
  uint8_t* tmp = static_cast<uint8_t*>(tmpv);
  const int T64 = (int)(np / 64);
  // the init may leave tiles unwritten only when every first product is masked by the
  // map (masks hold 64 chunks of 128: K = s <= 8192)
  const uint8_t* init_nz = (nz && np <= 16384) ? nz : nullptr;
  hipLaunchKernelGGL(tri_init_bf16x6_kernel, dim3(T64, T64, count), dim3(256), 0, stream, L, Dinv, np, T, Tt, sL,
                     sD, sT, sTt, skip, init_nz, snz, (int)(np / 64));
  if (hipGetLastError() != hipSuccess) return -2;
  // element offsets inside the split copies: sub-matrices start at multiples of 128
  // columns, so byte offset = 6 x element offset
  const int64_t n = np;
  for (int64_t s = 128; s < n; s *= 2) {
    const int64_t gs = 6 * 2 * s * (np + 1);  // group stride inside T and Tt, bytes
    const int full = (int)(n / (2 * s));
    int rc;
    if (full > 0) {
      // tmp^T = (T21 V11)^T, one s x s tmp^T per group
      rc = launch_tri6(stream, 1, (int)s, (int)s, (int)s, 1.f, T + 6 * s * np, np, Tt, np, nullptr, 0, tmp, s, full,
                       gs, gs, 0, 6 * s * s, count, sT, sTt, 0, sTmp, skip, zr, (int)s, 0, (int)(2 * s), (int)s);
      if (rc) return rc;
      // V21 = -V22 tmp into T21 and, transposed, into Tt
      rc = launch_tri6(stream, 2, (int)s, (int)s, (int)s, -1.f, T + 6 * s * (np + 1), np, tmp, s, T + 6 * s * np, np,
                       Tt + 6 * s, np, full, gs, 6 * s * s, gs, gs, count, sT, sTmp, sT, sTt, skip, zr, (int)s, 0,
                       (int)(2 * s), (int)s);
      if (rc) return rc;
    }
    const int64_t base = (int64_t)full * 2 * s;
    const int64_t n2 = n - base - s;
    if (n2 > 0) {
      rc = launch_tri6(stream, 1, (int)n2, (int)s, (int)s, 1.f, T + 6 * ((base + s) * np + base), np,
                       Tt + 6 * (base * np + base), np, nullptr, 0, tmp, n2, 1, 0, 0, 0, 0, count, sT, sTt, 0, sTmp,
                       skip, zr, (int)(base + s), (int)base, 0, (int)s);
      if (rc) return rc;
      rc = launch_tri6(stream, 2, (int)n2, (int)s, (int)n2, -1.f, T + 6 * (base + s) * (np + 1), np, tmp, n2,
                       T + 6 * ((base + s) * np + base), np, Tt + 6 * (base * np + base + s), np, 1, 0, 0, 0, 0, count,
                       sT, sTmp, sT, sTt, skip, zr, (int)(base + s), (int)base, 0, (int)s);
      if (rc) return rc;
    }
  }
  return 0;
}

}  // namespace glasso
