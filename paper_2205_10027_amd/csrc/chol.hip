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
constexpr int OUTER = 1024;    // outer panel width of the blocked Cholesky
constexpr int MID = 512;       // middle panel width: its blocks update each other first
constexpr int LEFT_MIN_N = 2048;  // left-looking leaf steps above this padded size

// One step of the blocked Cholesky: the 128-column block whose diagonal block is at
// A, with `rest` rows of the panel below it (a multiple of 64).
//
// Every workgroup factors the diagonal block in LDS (lds_potrf); all of them
// compute identical values.  Workgroup 0 writes diag(L) to dL and the strict lower
// part of L11 transposed into the strict upper triangle of the block: the lower
// triangle is still being read by the other workgroups, so finish_diag_blocks
// moves L11 into place after the whole factorisation (and inverts it there).
// Workgroup 1 + q solves rows 64q .. 64q + 63 of the panel below,
// L21 = A21 inv(L11)^T, in place: it owns those rows entirely.  k0 is the block's
// global column, used to report the first failing pivot.
//
// The solve works on the transpose, X^T = inv(L11) R^T, in 16-column blocks b:
//   Y_b^T = R_b^T - sum_{q<b} L_bq X_q^T,   X_b^T = inv(L_bb) Y_b^T,
// with the inverses of the eight 16x16 diagonal blocks computed first.  In the
// v_mfma_f64_16x16x4f64 layouts the output block X_q^T (element (i, j) in lane
// j + 16 (i%4), register i/4) is exactly the B operand of the k-steps over its
// 16 rows, so every X_q stays in registers until the store.
//
// Left-looking inside a middle panel: the block column first receives the products
// of the kl panels to its left in the same middle panel (columns k0 - 128 kl ..
// k0), A_kk -= L_kp L_kp^T and, in each solving workgroup, R -= L_rp L_kp^T for its
// rows, panel by panel in 64-column halves staged through LDS.  Products of 16x16
// blocks that are zero are skipped, and with a zero-block map so are whole panels
// whose block-column rows (or the workgroup's rows) are zero: for banded factors
// only the adjacent panel's corner remains.  (Earlier middle panels reach the block
// through the right-looking updates of potrf_lower.)
__global__ __launch_bounds__(256) void leaf_potrf_kernel(double* A, int64_t lda, int k0, int rest, int kl,
                                                         double* dL, int* info, FactorBatch fb) {
  // problem blockIdx.y of the batch
  A += blockIdx.y * fb.sA;
  dL += blockIdx.y * fb.sdL;
  info += blockIdx.y;
  if (*info) return;
  __shared__ double a[NB][LDL];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool solver = blockIdx.x > 0 && rest > 0;

  // zero-block map bytes of the kl (at most MID / NB - 1) panels to the left: lane
  // 3 (kp - 1) + w of each wave loads byte w of panel k0 / NB - kp (w = 0, 1: the
  // block's two 64-row chunks; 2: this workgroup's rows), in one load issued with
  // the block's; combined into bits 2kp - 2 and 2kp - 1 (a bit per 64-column half)
  // of mA0, mA1 and mR
  const uint8_t* nzf = fb.nz ? fb.nz + blockIdx.y * fb.snz : nullptr;
  constexpr int KLMAX = MID / NB - 1;
  const bool use_map = nzf != nullptr && kl > 0;
  unsigned int mbv = 0u;
  if (use_map && lane < 3 * KLMAX) {
    const int kp = lane / 3 + 1, w = lane % 3;
    const int chunk = (w == 2 && solver) ? (k0 + NB) / 64 + (int)blockIdx.x - 1 : k0 / 64 + (w == 1 ? 1 : 0);
    mbv = nzf[(int64_t)max(k0 / NB - kp, 0) * fb.nz_chunks + chunk];
  }

  // rows of the panel owned by this wave: R[16 wave + i][.] in the layout of Y_b^T
  // with the in-block index permuted (register s of lane l: R[l%16][16b + 4(l/16) + s],
  // four consecutive columns per lane: two 16-byte loads per block, whole 128-byte
  // lines per row); issued first, they arrive while the block is loaded and factored
  const double* R = A + (int64_t)(NB + 64 * ((int)blockIdx.x - 1) + 16 * wave + (lane & 15)) * lda + 4 * (lane >> 4);
  v4d x[8];
  if (solver) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const double2 lo = *reinterpret_cast<const double2*>(R + 16 * b);
      const double2 hi = *reinterpret_cast<const double2*>(R + 16 * b + 2);
      x[b] = (v4d){lo.x, lo.y, hi.x, hi.y};
    }
  }

  // 32 independent 16-byte loads per thread (a wave reads 4 rows of 1 KB), all in
  // flight together
#pragma unroll
  for (int i = 0; i < NB * NB / 512; ++i) {
    const int e = 2 * (tid + 256 * i);
    const int r = e >> 7, c = e & 127;
    const double2 v = *reinterpret_cast<const double2*>(A + (int64_t)r * lda + c);
    a[r][c] = (c <= r) ? v.x : 0.0;
    a[r][c + 1] = (c + 1 <= r) ? v.y : 0.0;
  }
  __syncthreads();
  unsigned int mA0 = 0xffu, mA1 = 0xffu, mR = solver ? 0xffu : 0u;
  if (use_map) {
    mA0 = mA1 = mR = 0u;
#pragma unroll
    for (int kp = 1; kp <= KLMAX; ++kp) {
      const unsigned int on = kp <= kl ? 3u : 0u;
      mA0 |= ((unsigned int)__builtin_amdgcn_readlane((int)mbv, 3 * kp - 3) & on) << (2 * kp - 2);
      mA1 |= ((unsigned int)__builtin_amdgcn_readlane((int)mbv, 3 * kp - 2) & on) << (2 * kp - 2);
      mR |= ((unsigned int)__builtin_amdgcn_readlane((int)mbv, 3 * kp - 1) & (solver ? on : 0u)) << (2 * kp - 2);
    }
  }

  const int li = lane & 15, lk = lane >> 4;
  // The solve's MFMA products run with the index inside every 16-block permuted,
  // t -> pt(t) = 4 (t mod 4) + t / 4, for the L11 rows (A operand) and the X^T rows
  // (B operand and result): result register r of lane l then holds original row
  // 4 (l/16) + r, so each lane keeps four consecutive columns of its row of X.  The
  // products are the same sums in the same k order.
  const int pli = 4 * (li & 3) + (li >> 2);
  // nonzero 16x16 blocks (b, q) of a staged 128 x 64 half panel, bit 4b + q; two
  // masks used in turn, the next one cleared while the current one is in use
  __shared__ unsigned int dmask[2];
  auto left_updates = [&](v4d(&acc)[9], const int(&bi)[9], const int(&bj)[9]) {
    int phase = 0;
    for (int kp = kl; kp >= 1; --kp) {
      // map bits of panel k0 / NB - kp: bit h = a nonzero in columns 64h .. 64h + 63
      const int m0 = (mA0 >> (2 * kp - 2)) & 3, m1 = (mA1 >> (2 * kp - 2)) & 3, mr = (mR >> (2 * kp - 2)) & 3;
      if (!(m0 | m1)) continue;  // L_kp = 0: nothing to subtract
      const double* D = A - NB * kp;  // L_kp: rows k0.., columns of panel P
      const double* Rr = A + (int64_t)(NB + 64 * ((int)blockIdx.x - 1) + 16 * wave + li) * lda - NB * kp;
#pragma unroll 1
      for (int h = 0; h < 2; ++h) {
        const bool d0 = (m0 >> h) & 1, d1 = (m1 >> h) & 1;
        if (!(d0 || d1)) continue;
        const bool rows_h = (mr >> h) & 1;
        unsigned int* const mcur = &dmask[phase & 1];
        if (tid == 0) dmask[(phase + 1) & 1] = 0u;
        // stage L_kp[:, 64h .. 64h + 63] (a 64-row chunk that the map shows zero is
        // staged as zeros) and collect the nonzero 16x16 blocks: thread t holds
        // columns 2t mod 64 and 2t mod 64 + 1 of rows t/32 + 8i.  The loads are
        // unconditional (every row is inside the matrix), so all sixteen are in
        // flight together.
        unsigned int bits = 0u;
        const int c = (2 * tid) & 63, r0 = tid >> 5;
        double2 vv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) vv[i] = *reinterpret_cast<const double2*>(D + (int64_t)(r0 + 8 * i) * lda + 64 * h + c);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int r = r0 + 8 * i;
          const bool keep = i < 8 ? d0 : d1;
          const double2 v = keep ? vv[i] : make_double2(0.0, 0.0);
          a[r][c] = v.x;
          a[r][c + 1] = v.y;
          if (v.x != 0.0 || v.y != 0.0) bits |= 1u << (4 * (r >> 4) + (c >> 4));
        }
        if (bits) atomicOr(mcur, bits);
        // this wave's 16 rows of L_rp, in the B layout: rp[q][s] = row li, column 16q + 4s + lk
        double rp[4][4];
        if (rows_h) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) rp[q][s2] = Rr[64 * h + 16 * q + 4 * s2 + lk];
        }
        __syncthreads();
        const unsigned int dm = *mcur;
        // A_kk -= L_kp L_kp^T on this wave's blocks of the lower triangle, the nine
        // accumulators in turn between dependent MFMAs
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bool on[9];
#pragma unroll
          for (int sl = 0; sl < 9; ++sl)
            on[sl] = bj[sl] >= 0 && ((dm >> (4 * bi[sl] + q)) & 1u) && ((dm >> (4 * bj[sl] + q)) & 1u);
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
            for (int sl = 0; sl < 9; ++sl)
              if (on[sl])
                acc[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[16 * bi[sl] + li][16 * q + 4 * s2 + lk],
                                                             a[16 * bj[sl] + li][16 * q + 4 * s2 + lk], acc[sl], 0,
                                                             0, 0);
        }
        // R^T -= L_kp L_rp^T: block b of Y^T from block (b, q) of L_kp and slice q of rp
        if (rows_h) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool rq = __ballot((rp[q][0] != 0.0) || (rp[q][1] != 0.0) || (rp[q][2] != 0.0) ||
                                     (rp[q][3] != 0.0)) != 0;
            if (!rq) continue;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
              for (int b = 0; b < 8; ++b)
                if ((dm >> (4 * b + q)) & 1u)
                  x[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[16 * b + pli][16 * q + 4 * s2 + lk], rp[q][s2],
                                                              x[b], 0, 0, 0);
          }
        }
        ++phase;
        __syncthreads();  // before the next half overwrites the staging
      }
    }
  };
  if (tid == 0) {
    dmask[0] = 0u;
    dmask[1] = 0u;
  }
  const int fail = kl > 0 ? lds_potrf<NB>(a, tid, left_updates) : lds_potrf<NB>(a, tid);
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
    return;
  }
  if (!solver) return;

  // inverses of the 16x16 diagonal blocks: wave w inverts block 2w in lanes 0..15
  // and block 2w + 1 in lanes 32..47, lane c computing column c by forward
  // substitution, column-oriented: once x_k is known it is subtracted from every
  // later row (each row still sums its terms in k order), so the dependent chain is
  // one step per row, not one per term.  1/L_ii: the hardware reciprocal refined by
  // one third-order step.  The inverses go to the free strict upper triangle: block
  // b < 7 at tile (b, 7), block 7 at tile (0, 6) (16x16 tiles).
  {
    const int c = lane & 31, b = 2 * wave + (lane >> 5), o = 16 * b;
    if (c < 16) {
      double rd[16], xv[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const double d = a[o + i][o + i];
        const double q0 = __builtin_amdgcn_rcp(d);
        const double e = fma(-d, q0, 1.0);
        rd[i] = fma(q0, fma(e, e, e), q0);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) xv[i] = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        xv[k] = xv[k] * rd[k];
#pragma unroll
        for (int i = k + 1; i < 16; ++i) xv[i] -= a[o + i][o + k] * xv[k];
      }
      const int r0 = (b < 7) ? o : 0, c0 = (b < 7) ? 112 : 96;
#pragma unroll
      for (int i = 0; i < 16; ++i) a[r0 + i][c0 + c] = xv[i];
    }
  }
  __syncthreads();

#pragma unroll
  for (int q = 0; q < 8; ++q) {
    // a block Y_q^T that is zero in the whole wave gives X_q = 0 and changes no later
    // block (banded factors: the rows below reach only the last columns of L11)
    const bool live = __ballot((x[q][0] != 0.0) || (x[q][1] != 0.0) || (x[q][2] != 0.0) || (x[q][3] != 0.0)) != 0;
    if (!live) continue;
    // X_q^T = inv(L_qq) Y_q^T
    const int r0 = (q < 7) ? 16 * q : 0, c0 = (q < 7) ? 112 : 96;
    v4d xq = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      xq = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r0 + pli][c0 + 4 * lk + s], x[q][s], xq, 0, 0, 0);
    x[q] = xq;
    // Y_b^T -= L_bq X_q^T for the later blocks
#pragma unroll
    for (int b = q + 1; b < 8; ++b)
#pragma unroll
      for (int s = 0; s < 4; ++s)
        x[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[16 * b + pli][16 * q + 4 * lk + s], x[q][s], x[b], 0, 0, 0);
  }
  // the solved rows go out through LDS so that each store writes a whole row
  // (1 KB per instruction) instead of 32 bytes in each of 16 rows
  __syncthreads();  // every wave is done reading L11 and the inverse blocks
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int s = 0; s < 4; ++s) a[16 * wave + li][16 * b + 4 * lk + s] = x[b][s];
  __syncthreads();
  double* const Rw = A + (int64_t)(NB + 64 * ((int)blockIdx.x - 1) + 16 * wave) * lda + 2 * lane;
#pragma unroll
  for (int r = 0; r < 16; ++r)
    *reinterpret_cast<double2*>(Rw + (int64_t)r * lda) = make_double2(a[16 * wave + r][2 * lane], a[16 * wave + r][2 * lane + 1]);
  if (fb.nz) {
    // which halves of these 64 solved rows hold a nonzero (the updates skip zero
    // blocks): bit 0 columns 0..63, bit 1 columns 64..127
    bool nz0 = false, nz1 = false;
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (b < 4)
          nz0 = nz0 || x[b][s] != 0.0;
        else
          nz1 = nz1 || x[b][s] != 0.0;
      }
    // per-wave ballots combined through LDS: one barrier for both bits
    __shared__ unsigned int nzw[4];
    const uint64_t b0 = __ballot(nz0), b1 = __ballot(nz1);
    if (lane == 0) nzw[wave] = (b0 ? 1u : 0u) | (b1 ? 2u : 0u);
    __syncthreads();
    if (tid == 0)
      fb.nz[blockIdx.y * fb.snz + (int64_t)(k0 / NB) * fb.nz_chunks + (k0 + NB) / 64 + (int)blockIdx.x - 1] =
          (uint8_t)(nzw[0] | nzw[1] | nzw[2] | nzw[3]);
  }
}

// After the factorisation, one workgroup per 128x128 diagonal block: the strict
// lower part of the block from its transposed copy in the strict upper triangle,
// the diagonal from dL; then the inverse of the block (lds_trtri) to Dinv (ld 128,
// zeros above the diagonal).
__global__ __launch_bounds__(256) void finish_diag_blocks_kernel(double* A, int64_t lda, const double* dL,
                                                                 double* Dinv, const int* skip, FactorBatch fb) {
  if (skip && skip[blockIdx.y]) return;
  double* D = A + blockIdx.y * fb.sA + (int64_t)blockIdx.x * NB * (lda + 1);
  const double* d = dL + blockIdx.y * fb.sdL + (int64_t)blockIdx.x * NB;
  double* Di = Dinv + blockIdx.y * fb.sDinv + (int64_t)blockIdx.x * NB * NB;
  __shared__ double a[NB][LDL];
  const int tid = threadIdx.x;
  // row r of the stored block holds L[c][r] for c > r
#pragma unroll 8
  for (int i = 0; i < NB * NB / 512; ++i) {
    const int e = 2 * (tid + 256 * i);
    const int r = e >> 7, c = e & 127;
    const double2 v = *reinterpret_cast<const double2*>(D + (int64_t)r * lda + c);
    a[c][r] = (c > r) ? v.x : 0.0;
    a[c + 1][r] = (c + 1 > r) ? v.y : 0.0;
  }
  __syncthreads();
  if (tid < NB) a[tid][tid] = d[tid];
  __syncthreads();
#pragma unroll 8
  for (int i = 0; i < NB * NB / 256; ++i) {
    const int e = tid + 256 * i;
    const int r = e >> 7, c = e & 127;
    if (c <= r) D[(int64_t)r * lda + c] = a[r][c];
  }
  lds_trtri<NB>(a, tid);
#pragma unroll 8
  for (int i = 0; i < NB * NB / 256; ++i) {
    const int e = tid + 256 * i;
    const int r = e >> 7, c = e & 127;
    Di[e] = (c <= r) ? a[r][c] : 0.0;
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

int finish_factor(hipStream_t stream, double* A, int64_t lda, int n, const double* dL, double* Dinv,
                  const int* skip, const FactorBatch& fb) {
  if (n % NB) return -1;
  if (fb.count <= 0) return 0;
  hipLaunchKernelGGL(finish_diag_blocks_kernel, dim3(n / NB, fb.count), dim3(256), 0, stream, A, lda, dL, Dinv, skip,
                     fb);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int potrf_lower(hipStream_t stream, double* A, int64_t lda, int n, double* dL, double* Dinv, int* info,
                const FactorBatch& fb, int finish, LeafTimer* timer) {
  if (n % NB) return -1;
  if (fb.count <= 0) return 0;
  ZBatch zA;  // operands and output inside the factored matrix
  zA.count = fb.count;
  zA.sA = zA.sB = zA.sC = fb.sA;
  zA.nz = fb.nz;
  zA.snz = fb.snz;
  zA.nz_chunks = fb.nz_chunks;
  // the updates' operands: rows from r of the panels from column c
  auto rows = [&](int r, int c) {
    ZBatch z = zA;
    z.nz_row0 = z.nz_col0 = r;
    z.nz_k0 = c;
    return z;
  };
  // Inside a middle panel the blocks update each other left-looking, in the leaf
  // steps, above LEFT_MIN_N: there a leaf launch has enough workgroups (one per 64
  // rows below the block) that its own K <= 384 update costs less than a separate
  // K = 128 launch per step.  Below it the middle panel is updated right-looking.
  const bool left_looking = n > LEFT_MIN_N;
  int rc = 0;
  for (int K0 = 0; K0 < n && rc == 0; K0 += OUTER) {
    const int K1 = min(K0 + OUTER, n);
    for (int M0 = K0; M0 < K1 && rc == 0; M0 += MID) {
      const int M1 = min(M0 + MID, K1);
      for (int k = M0; k < M1 && rc == 0; k += NB) {
        // factor the diagonal block and solve the panel below it (L21 = A21 inv(L11)^T)
        double* Akk = A + (int64_t)k * lda + k;
        const int rest = n - k - NB;
        const bool timed = timer && timer->used + 2 <= timer->cap && k < timer->n;
        if (timed && hipEventRecord(timer->ev[timer->used], stream) != hipSuccess) return -2;
        // panels to the left in this middle panel, applied inside the leaf step
        const int kl = left_looking ? (k - M0) / NB : 0;
        hipLaunchKernelGGL(leaf_potrf_kernel, dim3(1 + rest / 64, fb.count), dim3(256), 0, stream, Akk, lda, k,
                           rest, kl, dL + k, info, fb);
        if (hipGetLastError() != hipSuccess) return -2;
        if (timed) {
          if (hipEventRecord(timer->ev[timer->used + 1], stream) != hipSuccess) return -2;
          timer->used += 2;
          const int64_t left = timer->n - k;
          const double nb = (double)(left < NB ? left : NB);
          const double below = (double)(left > NB ? left - NB : 0);
          // the block's left-looking update (K = 128 kl: the rows below, and the lower
          // half of the diagonal block), its factor and the panel solve
          const double kk = (double)(NB * kl);
          timer->flops += timer->active * (nb * nb * nb / 3.0 + below * nb * nb + 2.0 * below * nb * kk + nb * nb * kk);
        }
        if (!left_looking && k + NB < M1) {
          // right-looking: update of the remaining columns of the middle panel (K = 128)
          const double* Pk = A + (int64_t)(k + NB) * lda + k;
          rc = gemm_f64(stream, 0, 0, rest, M1 - k - NB, NB, -1.0, Pk, lda, Pk, lda, 1.0,
                        A + (int64_t)(k + NB) * lda + (k + NB), lda, 0, 0, 0, info, 1, 0, 0, 0, 0, rows(k + NB, k));
          if (rc) return rc;
        }
      }
      if (M1 < K1) {
        // the rest of the outer panel from the whole middle panel (K = M1 - M0)
        const double* Pm = A + (int64_t)M1 * lda + M0;
        rc = gemm_f64(stream, 0, 0, n - M1, K1 - M1, M1 - M0, -1.0, Pm, lda, Pm, lda, 1.0,
                      A + (int64_t)M1 * lda + M1, lda, 0, 0, 0, info, 1, 0, 0, 0, 0, rows(M1, M0));
        if (rc) return rc;
      }
    }
    if (K1 < n) {
      // trailing lower triangle: A22 -= L21 L21^T with K = panel width
      const double* L21 = A + (int64_t)K1 * lda + K0;
      rc = gemm_f64(stream, 0, 0, n - K1, n - K1, K1 - K0, -1.0, L21, lda, L21, lda, 1.0,
                    A + (int64_t)K1 * lda + K1, lda, 1, 0, 0, info, 1, 0, 0, 0, 0, rows(K1, K0));
    }
  }
  if (rc) return rc;
  return finish ? finish_factor(stream, A, lda, n, dL, Dinv, info, fb) : 0;
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
