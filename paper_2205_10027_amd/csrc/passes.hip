// HBM-bound elementwise passes of pISTA (FP64, gfx950) and their deterministic
// reductions.
//
// pass_grad  (Sec. 4.1, eqs. grad_hessian, free_set, M, G+; stopping rule of Sec. 6):
//   g = S - W, M = (A != 0) | (|g| > lam), G = sign(A) or -sign(g),
//   Z = (g + lam G) (.) M  -- the minimum-norm subgradient, the input of A Z A,
//   GM = G (.) M as int8 (both full symmetric), and sums for ||Z||_1, ||Z||_F, max|Z|, ||A||_1, nnz(A),
//   tr(SA); a one-workgroup kernel then forms KKT = ||Z||_1/||A||_1 and F(A).
// pass_trial (eqs. c, b, d_sol; Alg. 1 masked update):
//   C_ij = lam (A_ii A_jj + A_ij^2) (i != j), lam A_ii^2 (i = j);
//   B = P - C (.) GM with P = A Z A;  At = M (.) ST(A - tB, tC);
//   sums of S (.) (At - A) and |At| - |A| for the difference-form decrease.
//   G-ISTA mode (eq. proximal_gen with H = I): At = ST(A - t (S - W), t lam), with
//   sums of W (.) (At - A) and (At - A)^2 for its quadratic-bound test.
//
// Both passes visit only the tiles on or below the diagonal (64x64 tiles of the
// padded matrix), read lower triangles, and write symmetric outputs through an
// LDS transpose.  Off-diagonal elements carry weight 2 in every sum.
// Floating-point contraction is disabled so each element is computed with the
// same sequence of IEEE operations as the plain formulas.
#pragma clang fp contract(off)

#include <float.h>

#include "bf16.h"
#include "common.h"
#include "elementwise.h"
#include "kernels.h"

namespace glasso {

namespace {

// ------------------------------------------------------------------ gradient pass
__global__ __launch_bounds__(256) void pass_grad_kernel(const double* __restrict__ S,
                                                        const double* __restrict__ W,
                                                        const double* __restrict__ A,
                                                        const double* __restrict__ dL, int64_t n,
                                                        int64_t np, double lam, double* __restrict__ Z,
                                                        uint8_t* __restrict__ Zs, int64_t sZs,
                                                        int8_t* __restrict__ GM, double* part, int T, PassBatch pb,
                                                        const double* __restrict__ Aprev) {
  __shared__ double zt[64][65];
  __shared__ int8_t gt[64][68];
  __shared__ double sh[4];
  const int pbi = blockIdx.y;
  if (pb.skip && pb.skip[pbi]) return;
  if (pb.lam) lam = pb.lam[pbi];
  S += pbi * pb.sS;
  W += pbi * pb.sM;
  A += pbi * pb.sM;
  if (Z) Z += pbi * pb.sM;
  if (Zs) Zs += pbi * sZs;
  GM += pbi * pb.sM;
  if (Aprev) Aprev += pbi * pb.sM;
  part += (int64_t)pbi * gridDim.x * GRAD_PARTS;
  int ti, tj;
  lower_tile(xcd_remap(blockIdx.x, gridDim.x), T, ti, tj);
  const int tid = threadIdx.x, c = tid & 63, rw = tid >> 6;
  const int64_t i0 = (int64_t)ti * 64, j0 = (int64_t)tj * 64;
  const bool diag = (ti == tj);

  double s_absz = 0.0, s_z2 = 0.0, m_absz = 0.0, s_absa = 0.0, s_nnz = 0.0, s_sa = 0.0, s_dw = 0.0;
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int r = rw + 4 * q;
    const int64_t i = i0 + r, j = j0 + c;
    const int64_t off = i * np + j;
    double z = 0.0;
    int8_t gm = 0;
    if (!diag || c <= r) {
      if (i < n && j < n) {
        const double a = A[off], s = S[off], w = W[off];
        grad_element(a, s, w, lam, z, gm);
        const bool nz = (a != 0.0);
        const double wgt = (i == j) ? 1.0 : 2.0;
        s_absz += wgt * fabs(z);
        s_z2 += wgt * (z * z);
        m_absz = fmax(m_absz, fabs(z));
        s_absa += wgt * fabs(a);
        s_nnz += nz ? wgt : 0.0;
        s_sa += wgt * (s * a);
        if (Aprev) s_dw += wgt * (w * (a - Aprev[off]));
      }
      if (Z) Z[off] = z;
      if (Zs) store_split2(Zs, np, i, j, z);
      GM[off] = gm;
    }
    zt[r][c] = z;
    gt[r][c] = gm;
  }
  __syncthreads();
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int r = rw + 4 * q;
    if (!diag) {
      if (Z) Z[(j0 + r) * np + i0 + c] = zt[c][r];
      if (Zs) store_split2(Zs, np, j0 + r, i0 + c, zt[c][r]);
      GM[(j0 + r) * np + i0 + c] = gt[c][r];
    } else if (c > r) {
      if (Z) Z[(i0 + r) * np + j0 + c] = zt[c][r];
      if (Zs) store_split2(Zs, np, i0 + r, j0 + c, zt[c][r]);
      GM[(i0 + r) * np + j0 + c] = gt[c][r];
    }
  }

  const double b0 = block_sum(s_absz, sh);
  const double b1 = block_sum(s_z2, sh);
  const double b2 = block_max(m_absz, sh);
  const double b3 = block_sum(s_absa, sh);
  const double b4 = block_sum(s_nnz, sh);
  const double b5 = block_sum(s_sa, sh);
  const double b6 = block_sum(s_dw, sh);
  if (tid == 0) {
    double* pp = part + (int64_t)blockIdx.x * GRAD_PARTS;
    pp[0] = b0;
    pp[1] = b1;
    pp[2] = b2;
    pp[3] = b3;
    pp[4] = b4;
    pp[5] = b5;
    pp[6] = b6;
  }
}

// fixed-order reduction of the gradient-pass partials, then KKT and F(A)
__global__ __launch_bounds__(256) void finish_grad_kernel(const double* part, int nparts, const double* dL,
                                                          int64_t nlog, double lam, double* scal, PassBatch pb) {
  __shared__ double sh[4];
  const int tid = threadIdx.x;
  const int pbi = blockIdx.x;
  if (pb.skip && pb.skip[pbi]) return;
  if (pb.lam) lam = pb.lam[pbi];
  part += (int64_t)pbi * nparts * GRAD_PARTS;
  dL += pbi * pb.sV;
  scal += (int64_t)pbi * SC_COUNT;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0, t5 = 0.0, t6 = 0.0;
  for (int b = tid; b < nparts; b += 256) {
    const double* pp = part + (int64_t)b * GRAD_PARTS;
    t0 += pp[0];
    t1 += pp[1];
    t2 = fmax(t2, pp[2]);
    t3 += pp[3];
    t4 += pp[4];
    t5 += pp[5];
    t6 += pp[6];
  }
  double tl = 0.0;
  for (int64_t i = tid; i < nlog; i += 256) tl += log(dL[i]);
  const double sz = block_sum(t0, sh);
  const double sz2 = block_sum(t1, sh);
  const double mz = block_max(t2, sh);
  const double sa = block_sum(t3, sh);
  const double nnz = block_sum(t4, sh);
  const double ssa = block_sum(t5, sh);
  const double dwn = block_sum(t6, sh);
  const double ld = 2.0 * block_sum(tl, sh);
  if (tid == 0) {
    scal[SC_DW_NEW] = dwn;
    scal[SC_SUM_ABS_Z] = sz;
    scal[SC_SUM_Z2] = sz2;
    scal[SC_MAX_ABS_Z] = mz;
    scal[SC_SUM_ABS_A] = sa;
    scal[SC_NNZ_A] = nnz;
    scal[SC_SUM_SA] = ssa;
    scal[SC_LOGDET] = ld;
    scal[SC_OBJECTIVE] = -ld + ssa + lam * sa;
    scal[SC_KKT_REL1] = sz / sa;
    scal[SC_KKT_FRO] = sqrt(sz2);
  }
}

// ------------------------------------------------------------------ trial pass
__global__ __launch_bounds__(256) void pass_trial_kernel(const double* __restrict__ A,
                                                         const double* __restrict__ P,
                                                         const double* __restrict__ S,
                                                         const int8_t* __restrict__ GM, int64_t n, int64_t np,
                                                         double lam, double t, double* __restrict__ At,
                                                         double* __restrict__ Lt, double* part, int* info_reset,
                                                         int T, PassBatch pb, const double* __restrict__ W,
                                                         int gista) {
  __shared__ double tt[64][65];
  __shared__ double di[64], dj[64];
  __shared__ double sh[4];
  const int pbi = blockIdx.y, prob = pbi / pb.div;  // trial slot, its problem
  const bool skipped = pb.skip && pb.skip[pbi];
  if (blockIdx.x == 0 && threadIdx.x == 0) info_reset[pbi] = skipped ? -1 : 0;
  if (skipped) return;
  if (pb.lam) lam = pb.lam[prob];
  if (pb.t) t = pb.t[pbi];
  A += prob * pb.sM;
  P += prob * pb.sM;
  S += prob * pb.sS;
  GM += prob * pb.sM;
  if (W) W += prob * pb.sM;
  At += pbi * pb.sM;
  Lt += pbi * pb.sM;
  part += (int64_t)pbi * gridDim.x * TRIAL_PARTS;
  int ti, tj;
  lower_tile(xcd_remap(blockIdx.x, gridDim.x), T, ti, tj);
  const int tid = threadIdx.x, c = tid & 63, rw = tid >> 6;
  const int64_t i0 = (int64_t)ti * 64, j0 = (int64_t)tj * 64;
  const bool diag = (ti == tj);
  if (tid < 64)
    di[tid] = A[(i0 + tid) * (np + 1)];
  else if (tid < 128)
    dj[tid - 64] = A[(j0 + tid - 64) * (np + 1)];
  __syncthreads();

  double s_tr = 0.0, s_l1 = 0.0, s_nnz = 0.0, s_w = 0.0, s_d2 = 0.0;
  // the free-set flags of all 16 rows first (in-tile offsets are inside the padded
  // matrix; flags past n are not used): one round trip instead of one per row group
  int8_t gmv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) gmv[q] = GM[(i0 + rw + 4 * q) * np + j0 + c];
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int r = rw + 4 * q;
    const int64_t i = i0 + r, j = j0 + c;
    const int64_t off = i * np + j;
    double at = 0.0;
    if (!diag || c <= r) {
      if (i < n && j < n) {
        // off the free set A_ij = 0 and At_ij = 0: nothing else to read
        const int8_t gm = gmv[q];
        if (gm != 0) {
          const double a = A[off];
          const double s = S[off];
          if (gista) {
            at = gista_element(a, s, W[off], lam, t);
          } else {
            const double p = P[off];
            const double Cij = c_element(i == j, di[r], dj[c], a, lam);
            at = trial_element(a, p, Cij, (double)gm, t);
          }
          const double wgt = (i == j) ? 1.0 : 2.0;
          const double d = at - a;
          s_tr += wgt * (s * d);
          s_l1 += wgt * (fabs(at) - fabs(a));
          s_nnz += (at != 0.0) ? wgt : 0.0;
          s_d2 += wgt * (d * d);
          if (W) s_w += wgt * (W[off] * d);
        }
      } else {
        at = (i == j) ? 1.0 : 0.0;
      }
      At[off] = at;
      Lt[off] = at;
    }
    tt[r][c] = at;
  }
  __syncthreads();
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int r = rw + 4 * q;
    if (!diag)
      At[(j0 + r) * np + i0 + c] = tt[c][r];
    else if (c > r)
      At[(i0 + r) * np + j0 + c] = tt[c][r];
  }
  const double b0 = block_sum(s_tr, sh);
  const double b1 = block_sum(s_l1, sh);
  const double b2 = block_sum(s_nnz, sh);
  const double b3 = block_sum(s_w, sh);
  const double b4 = block_sum(s_d2, sh);
  if (tid == 0) {
    double* pp = part + (int64_t)blockIdx.x * TRIAL_PARTS;
    pp[0] = b0;
    pp[1] = b1;
    pp[2] = b2;
    pp[3] = b3;
    pp[4] = b4;
  }
}

// After the trial's Cholesky: dF = 2 sum log(L_ii / Lt_ii) + sum S(At-A) + lam sum(|At|-|A|),
// and the G-ISTA bound excess 2 sum log(L_ii / Lt_ii) + sum W(At-A) - ||At-A||^2 / (2t).
__global__ __launch_bounds__(256) void finish_trial_kernel(const double* part, int nparts, const double* dL,
                                                           const double* dLt, const int* info, int64_t n,
                                                           double lam, double* scal, PassBatch pb, double t) {
  __shared__ double sh[4];
  const int tid = threadIdx.x;
  const int pbi = blockIdx.x, prob = pbi / pb.div;  // trial slot, its problem
  if (pb.skip && pb.skip[pbi]) return;
  if (pb.lam) lam = pb.lam[prob];
  if (pb.t) t = pb.t[pbi];
  part += (int64_t)pbi * nparts * TRIAL_PARTS;
  dL += prob * pb.sV;
  dLt += pbi * pb.sV;
  scal += (int64_t)pbi * SC_COUNT;
  const int inf = info[pbi];
  double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0, tl = 0.0;
  for (int b = tid; b < nparts; b += 256) {
    t0 += part[(int64_t)b * TRIAL_PARTS + 0];
    t1 += part[(int64_t)b * TRIAL_PARTS + 1];
    t2 += part[(int64_t)b * TRIAL_PARTS + 2];
    t3 += part[(int64_t)b * TRIAL_PARTS + 3];
    t4 += part[(int64_t)b * TRIAL_PARTS + 4];
  }
  if (inf == 0)
    for (int64_t i = tid; i < n; i += 256) tl += log(dL[i] / dLt[i]);
  const double dtr = block_sum(t0, sh);
  const double dl1 = block_sum(t1, sh);
  const double nnz = block_sum(t2, sh);
  const double dw = block_sum(t3, sh);
  const double d2 = block_sum(t4, sh);
  const double dlog = 2.0 * block_sum(tl, sh);
  if (tid == 0) {
    scal[SC_DW] = dw;
    scal[SC_D2] = d2;
    scal[SC_QB] = (dlog + dw) - d2 / (2.0 * t);
    scal[SC_DTR] = dtr;
    scal[SC_DL1] = dl1;
    scal[SC_DLOG] = dlog;
    scal[SC_DF] = dlog + dtr + lam * dl1;
    scal[SC_TRIAL_INFO] = (double)inf;
    scal[SC_NNZ_AT] = nnz;
    // <g, At - A> = sum S (.) (At - A) - sum W (.) (At - A), g = S - W
    scal[SC_PRED] = (dtr - dw) + lam * dl1;
  }
}

// ------------------------------------------------------------------ copies
__global__ void copy_in_kernel(const double* __restrict__ src, int64_t n, double* __restrict__ dst, int64_t np,
                               unsigned long long* bad, double lam, int check) {
  const int64_t total = np * np;
  unsigned long long nbad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / np, j = e - i * np;
    double v = 0.0;
    if (i < n && j < n) {
      v = src[i * n + j];
      if (check && j <= i) {
        if (!(fabs(v) <= DBL_MAX)) ++nbad;
        if (i == j && !(v + lam > 0.0)) ++nbad;
      }
    }
    dst[e] = v;
  }
  if (check && nbad) atomicAdd(bad, nbad);
}

// A^(0) = diag(1/(S_ii + lam)) with identity padding and, because it is diagonal,
// its factor and inverse in closed form: L = diag(sqrt(A_ii)) (diag(L) also in dL),
// the 128x128 diagonal-block inverses of L in Dinv (np x 128), W = diag(1/A_ii).
__device__ __forceinline__ double initial_diag(const double* Sp, int64_t n, int64_t np, double lam, int64_t i) {
  return (i < n) ? 1.0 / (Sp[i * np + i] + lam) : 1.0;
}
__global__ void init_diag_kernel(const double* __restrict__ Sp, int64_t n, int64_t np, double lam,
                                 double* __restrict__ A, double* __restrict__ L, double* __restrict__ dL,
                                 double* __restrict__ Dinv, double* __restrict__ W) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = np * np;
  for (int64_t e = first; e < total; e += stride) {
    const int64_t i = e / np, j = e - i * np;
    const double a = (i == j) ? initial_diag(Sp, n, np, lam, i) : 0.0;
    A[e] = a;
    L[e] = (i == j) ? sqrt(a) : 0.0;
    W[e] = (i == j) ? 1.0 / a : 0.0;
  }
  for (int64_t e = first; e < np * 128; e += stride) {
    const int64_t i = e >> 7;
    Dinv[e] = ((e & 127) == (i & 127)) ? 1.0 / sqrt(initial_diag(Sp, n, np, lam, i)) : 0.0;
  }
  for (int64_t i = first; i < np; i += stride) dL[i] = sqrt(initial_diag(Sp, n, np, lam, i));
}

// P = A Z A for a diagonal A: P_ij = (A_ii Z_ij) A_jj, rounded as the FP64 GEMM
// pair rounds it (X = A Z, then X A), for the problems with skip == 0.  64x64
// tiles; the tile's 128 diagonal entries are staged in LDS first.
__global__ __launch_bounds__(256) void diag_product_kernel(const double* __restrict__ A,
                                                           const double* __restrict__ Z, double* __restrict__ P,
                                                           int64_t np, int64_t sM, const int* skip) {
  if (skip && skip[blockIdx.z]) return;
  A += blockIdx.z * sM;
  Z += blockIdx.z * sM;
  P += blockIdx.z * sM;
  __shared__ double di[64], dj[64];
  const int tid = threadIdx.x, c = tid & 63;
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  if (tid < 64)
    di[tid] = A[(i0 + tid) * (np + 1)];
  else if (tid < 128)
    dj[tid - 64] = A[(j0 + tid - 64) * (np + 1)];
  __syncthreads();
  for (int r = tid >> 6; r < 64; r += 4) {
    const int64_t e = (i0 + r) * np + j0 + c;
    const double x = di[r] * Z[e];
    P[e] = x * dj[c];
  }
}

// dst (np x np) <- src (n x n, ld n); outside the n x n block: identity when
// pad_diag, else zero.  dst2 (may be null) receives the same values.
__global__ void pad_copy_f64_kernel(const double* __restrict__ src, int64_t n, int64_t np, double* __restrict__ dst,
                                    double* __restrict__ dst2, int pad_diag) {
  const int64_t total = np * np;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / np, j = e - i * np;
    double v;
    if (i < n && j < n)
      v = src[i * n + j];
    else
      v = (pad_diag && i == j) ? 1.0 : 0.0;
    dst[e] = v;
    if (dst2) dst2[e] = v;
  }
}

__global__ void pad_copy_i8_kernel(const int8_t* __restrict__ src, int64_t n, int64_t np, int8_t* __restrict__ dst) {
  const int64_t total = np * np;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / np, j = e - i * np;
    dst[e] = (i < n && j < n) ? src[i * n + j] : (int8_t)0;
  }
}

__global__ void unpad_copy_i8_kernel(const int8_t* __restrict__ src, int64_t np, int8_t* __restrict__ dst, int64_t n) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e - i * n;
    dst[e] = src[i * np + j];
  }
}

// out = 2 sum_{i<n} log d_i
// X_b = I (np x np) for count problems at stride nn
__global__ __launch_bounds__(256) void fill_identity_kernel(double* X, int64_t np, int64_t nn, int count) {
  const int64_t total = nn * count;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = e % nn;
    X[e] = (o / np == o % np) ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(256) void sum_log_kernel(const double* d, int64_t n, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += log(d[i]);
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) *out = 2.0 * t;
}

// dst (n x n, ld n) <- src (np x np).  mode 0: plain copy; mode 1: src holds only
// its lower triangle and dst receives the symmetric matrix it stands for; mode 2:
// lower triangle of src, zeros above.
__global__ __launch_bounds__(256) void sym_copy_out_kernel(const double* __restrict__ src, int64_t np,
                                                           double* __restrict__ dst, int64_t n, int mode,
                                                           int Tn) {
  __shared__ double tt[64][65];
  const int bi = blockIdx.x / Tn, bj = blockIdx.x % Tn;
  const int tid = threadIdx.x, c = tid & 63, rw = tid >> 6;
  const int64_t i0 = (int64_t)bi * 64, j0 = (int64_t)bj * 64;
  if (mode == 0 || bi > bj) {
    for (int q = 0; q < 16; ++q) {
      const int r = rw + 4 * q;
      const int64_t i = i0 + r, j = j0 + c;
      if (i < n && j < n) dst[i * n + j] = src[i * np + j];
    }
    return;
  }
  if (mode == 2) {
    for (int q = 0; q < 16; ++q) {
      const int r = rw + 4 * q;
      const int64_t i = i0 + r, j = j0 + c;
      if (i < n && j < n) dst[i * n + j] = (j <= i) ? src[i * np + j] : 0.0;
    }
    return;
  }
  // read the mirrored (lower) tile (bj, bi) and transpose it
  for (int q = 0; q < 16; ++q) {
    const int r = rw + 4 * q;
    const int64_t i = j0 + r, j = i0 + c;  // element of tile (bj, bi)
    tt[r][c] = (i < np && j < np) ? src[i * np + j] : 0.0;
  }
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int r = rw + 4 * q;
    const int64_t i = i0 + r, j = j0 + c;
    if (i < n && j < n) {
      double v;
      if (bi == bj)
        v = (c <= r) ? tt[r][c] : tt[c][r];  // upper part of a diagonal tile mirrors (c, r)
      else
        v = tt[c][r];
      dst[i * n + j] = v;
    }
  }
}

// make a padded matrix symmetric from its lower triangle, in place
__global__ __launch_bounds__(256) void mirror_lower_kernel(double* M, int64_t np, int T) {
  __shared__ double tt[64][65];
  int ti, tj;
  lower_tile(blockIdx.x, T, ti, tj);
  const int tid = threadIdx.x, c = tid & 63, rw = tid >> 6;
  const int64_t i0 = (int64_t)ti * 64, j0 = (int64_t)tj * 64;
  for (int q = 0; q < 16; ++q) {
    const int r = rw + 4 * q;
    tt[r][c] = M[(i0 + r) * np + j0 + c];
  }
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int r = rw + 4 * q;
    if (ti != tj)
      M[(j0 + r) * np + i0 + c] = tt[c][r];
    else if (c > r)
      M[(i0 + r) * np + j0 + c] = tt[c][r];
  }
}

// y = M x, one wave per row
__global__ __launch_bounds__(256) void gemv_kernel(const double* __restrict__ M, int64_t np,
                                                   const double* __restrict__ x, double* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= np) return;
  const double* mr = M + row * np;
  double s = 0.0;
  for (int64_t j = lane; j < np; j += 64) s += mr[j] * x[j];
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// x = y / ||y|| over the first n entries (zeros beyond), out = ||y||
__global__ __launch_bounds__(256) void normalize_kernel(const double* __restrict__ y, double* __restrict__ x,
                                                        int64_t n, int64_t np, double* out, int init) {
  __shared__ double sh[4];
  double s = 0.0;
  if (!init)
    for (int64_t i = threadIdx.x; i < n; i += 256) s += y[i] * y[i];
  const double nrm = init ? sqrt((double)n) : sqrt(block_sum(s, sh));
  for (int64_t i = threadIdx.x; i < np; i += 256) x[i] = (i < n) ? (init ? 1.0 : y[i]) / nrm : 0.0;
  if (threadIdx.x == 0 && out) *out = nrm;
}

// ------------------------------------------------------------------ sample covariance
// Column means of Y (m x n, row-major: one sample per row), eq. empirical_cov: one
// workgroup per 64 columns, lane = column, the four waves summing every fourth row,
// then their partial sums in a fixed order.
__global__ __launch_bounds__(256) void column_mean_kernel(const double* __restrict__ Y, int64_t m, int64_t n,
                                                          double* __restrict__ mu) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (j < n)
    for (int64_t i = wave; i < m; i += 4) s += Y[i * n + j];
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && j < n) mu[j] = ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) / (double)m;
}

// Yp (mp x np) = Y - 1 mu^T (mu null: Y itself), zeros in the padding rows and columns
__global__ __launch_bounds__(256) void center_pad_kernel(const double* __restrict__ Y, int64_t m, int64_t n,
                                                         const double* __restrict__ mu, double* __restrict__ Yp,
                                                         int64_t mp, int64_t np) {
  const int64_t total = mp * np;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / np, j = e - i * np;
    double v = 0.0;
    if (i < m && j < n) v = mu ? Y[i * n + j] - mu[j] : Y[i * n + j];
    Yp[e] = v;
  }
}

// Accept trial slot j = accept[b] - 1 of every problem b with accept[b] != 0:
// A_b <- At_j, L_b <- Lt_j (np x np each), dL_b <- dLt_j (np).
__global__ void accept_kernel(const int* accept, double* A, const double* At, double* L, const double* Lt,
                              double* dL, const double* dLt, int64_t nn, int64_t np, double* Aprev) {
  const int b = blockIdx.y;
  const int j = accept[b] - 1;  // trial slot to take, or none
  if (j < 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dst = (int64_t)b * nn, src = (int64_t)j * nn;
  for (int64_t e = i0; e < nn; e += stride) {
    if (Aprev) Aprev[dst + e] = A[dst + e];
    A[dst + e] = At[src + e];
    L[dst + e] = Lt[src + e];
  }
  for (int64_t e = i0; e < np; e += stride) dL[(int64_t)b * np + e] = dLt[(int64_t)j * np + e];
}

}  // namespace

int column_mean(hipStream_t stream, const double* Y, int64_t m, int64_t n, double* mu) {
  hipLaunchKernelGGL(column_mean_kernel, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, stream, Y, m, n, mu);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int center_pad(hipStream_t stream, const double* Y, int64_t m, int64_t n, const double* mu, double* Yp, int64_t mp,
               int64_t np) {
  const int blocks = (int)std::min<int64_t>((mp * np + 255) / 256, 16384);
  hipLaunchKernelGGL(center_pad_kernel, dim3(blocks), dim3(256), 0, stream, Y, m, n, mu, Yp, mp, np);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int accept_trials(hipStream_t stream, const int* accept, int count, double* A, const double* At, double* L,
                  const double* Lt, double* dL, const double* dLt, int64_t np, double* Aprev) {
  const int64_t nn = np * np;
  const int blocks = (int)std::min<int64_t>((nn + 255) / 256, 4096);
  hipLaunchKernelGGL(accept_kernel, dim3(blocks, count), dim3(256), 0, stream, accept, A, At, L, Lt, dL, dLt, nn, np,
                     Aprev);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int copy_in_padded(hipStream_t stream, const double* src, int64_t n, double* dst, int64_t np,
                   int64_t* bad_count_dev, double lam, int check) {
  const int64_t total = np * np;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(copy_in_kernel, dim3(blocks), dim3(256), 0, stream, src, n, dst, np,
                     reinterpret_cast<unsigned long long*>(bad_count_dev), lam, check);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int init_diag(hipStream_t stream, const double* Sp, int64_t n, int64_t np, double lam, double* A, double* L,
              double* dL, double* Dinv, double* W) {
  const int64_t total = np * np;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(init_diag_kernel, dim3(blocks), dim3(256), 0, stream, Sp, n, np, lam, A, L, dL, Dinv, W);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

static int grid_for(int64_t total) { return (int)std::min<int64_t>((total + 255) / 256, 16384); }

int diag_product(hipStream_t stream, const double* A, const double* Z, double* P, int64_t np, int count,
                 const int* skip) {
  if (count <= 0 || np % 64) return count <= 0 ? 0 : -1;
  const int T = (int)(np / 64);
  hipLaunchKernelGGL(diag_product_kernel, dim3(T, T, count), dim3(256), 0, stream, A, Z, P, np, np * np, skip);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int pad_copy_f64(hipStream_t stream, const double* src, int64_t n, int64_t np, double* dst, double* dst2,
                 int pad_diag) {
  hipLaunchKernelGGL(pad_copy_f64_kernel, dim3(grid_for(np * np)), dim3(256), 0, stream, src, n, np, dst, dst2,
                     pad_diag);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int pad_copy_i8(hipStream_t stream, const int8_t* src, int64_t n, int64_t np, int8_t* dst) {
  hipLaunchKernelGGL(pad_copy_i8_kernel, dim3(grid_for(np * np)), dim3(256), 0, stream, src, n, np, dst);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int unpad_copy_i8(hipStream_t stream, const int8_t* src, int64_t np, int8_t* dst, int64_t n) {
  hipLaunchKernelGGL(unpad_copy_i8_kernel, dim3(grid_for(n * n)), dim3(256), 0, stream, src, np, dst, n);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int fill_identity(hipStream_t stream, double* X, int64_t np, int count) {
  const int64_t total = np * np * count;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(fill_identity_kernel, dim3(blocks), dim3(256), 0, stream, X, np, np * np, count);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int sum_log(hipStream_t stream, const double* d, int64_t n, double* out) {
  hipLaunchKernelGGL(sum_log_kernel, dim3(1), dim3(256), 0, stream, d, n, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int pass_grad(hipStream_t stream, const double* S, const double* W, const double* A, const double* dL, int64_t n,
              int64_t nlog, int64_t np, double lam, double* Z, int8_t* GM, double* part, double* scal,
              const PassBatch& pb, void* Zs, int64_t sZs, const double* Aprev) {
  const int T = (int)(np / 64);
  const int tiles = T * (T + 1) / 2;
  hipLaunchKernelGGL(pass_grad_kernel, dim3(tiles, pb.count), dim3(256), 0, stream, S, W, A, dL, n, np, lam, Z,
                     static_cast<uint8_t*>(Zs), sZs, GM, part, T, pb, Aprev);
  hipLaunchKernelGGL(finish_grad_kernel, dim3(pb.count), dim3(256), 0, stream, part, tiles, dL, nlog, lam, scal, pb);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int pass_trial(hipStream_t stream, const double* A, const double* P, const double* S, const int8_t* GM, int64_t n,
               int64_t np, double lam, double t, double* At, double* Lt, double* part, int* info_reset,
               const PassBatch& pb, const double* W, int gista) {
  if (gista && !W) return -1;
  const int T = (int)(np / 64);
  const int tiles = T * (T + 1) / 2;
  hipLaunchKernelGGL(pass_trial_kernel, dim3(tiles, pb.count), dim3(256), 0, stream, A, P, S, GM, n, np, lam, t, At,
                     Lt, part, info_reset, T, pb, W, gista);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int finish_trial(hipStream_t stream, const double* part, int nparts, const double* dL, const double* dLt,
                 const int* info, int64_t n, double lam, double* scal, const PassBatch& pb, double t) {
  hipLaunchKernelGGL(finish_trial_kernel, dim3(pb.count), dim3(256), 0, stream, part, nparts, dL, dLt, info, n, lam,
                     scal, pb, t);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int sym_copy_out(hipStream_t stream, const double* src, int64_t np, double* dst, int64_t n, int mode) {
  const int Tn = (int)((n + 63) / 64);
  hipLaunchKernelGGL(sym_copy_out_kernel, dim3(Tn * Tn), dim3(256), 0, stream, src, np, dst, n, mode, Tn);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int mirror_lower(hipStream_t stream, double* M, int64_t np) {
  const int T = (int)(np / 64);
  hipLaunchKernelGGL(mirror_lower_kernel, dim3(T * (T + 1) / 2), dim3(256), 0, stream, M, np, T);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int power_iteration(hipStream_t stream, const double* M, int64_t n, int64_t np, double* vec, double* out, int iters) {
  double* x = vec;
  double* y = vec + np;
  hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(256), 0, stream, y, x, n, np, (double*)nullptr, 1);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(gemv_kernel, dim3((unsigned)((np + 3) / 4)), dim3(256), 0, stream, M, np, x, y);
    hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(256), 0, stream, y, x, n, np, out, 0);
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
