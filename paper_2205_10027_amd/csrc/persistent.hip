// Persistent solver for many small problems in one launch (n <= 64 each, sizes
// may differ).  Each workgroup starts with problem blockIdx.x and then takes the
// next untaken problem from a work queue (one atomic counter) until none is left,
// so problems that need many iterations do not hold up a fixed share of the
// others.  It runs the whole of Alg. 1 (Sec. 6 settings) for each on the device:
// factor, inverse, gradient pass and stopping test, A Z A, the backtracking line
// search with the cond-based fallback, and the accept step, with no host round
// trip.  FP64 throughout, with the same per-element formulas as the blocked passes.
//
// Per workgroup: the matrix being factored or inverted (64 x 65 doubles) and the
// A Z A operands (another 64 x 65) live in LDS; S, A, At, W, Z, P and the free-set
// signs of the current problem live in the workgroup's slot of a global workspace
// (L2-resident: 232 KB).  Every loop is bounded (max_iter iterations; trials stop
// once t < t_min), so every workgroup reaches its exit.
#pragma clang fp contract(off)
#include <float.h>

#include "common.h"
#include "elementwise.h"
#include "kernels.h"
#include "leaf.h"

namespace glasso {

namespace {

constexpr int SN = 64;       // padded edge
constexpr int SLD = SN + 1;  // LDS row stride
constexpr int SNN = SN * SN;

// W = V^T V for V = inv(L) lower in a (upper triangle of a is scratch): 16x16
// block (bi, bj), bi >= bj, sums k >= 16 bi with V[k][i] = 0 for k < i masked.
__device__ __forceinline__ v4d lauum_block(const double (*a)[SLD], int bi, int bj, int lane) {
  const int m = lane & 15, kk = lane >> 4;
  const int i = 16 * bi + m, j = 16 * bj + m;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k = 16 * bi; k < SN; k += 4) {
    const int kr = k + kk;
    const double x = (kr >= i) ? a[kr][i] : 0.0;  // A operand (m, k) = V[k][i]
    const double y = (kr >= j) ? a[kr][j] : 0.0;  // B operand (k, n) = V[k][j]
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
  }
  return acc;
}

// acc = X Y for 16x16 block (bi, bj): X(m, k) = x[16 bi + m][k], Y(k, n) = y[k][16 bj + n]
__device__ __forceinline__ v4d nn_block(const double (*x)[SLD], const double (*y)[SLD], int bi, int bj, int lane) {
  const int m = lane & 15, kk = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k = 0; k < SN; k += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[16 * bi + m][k + kk], y[k + kk][16 * bj + m], acc, 0, 0, 0);
  return acc;
}

// lower 16x16 block number job (0..9) of the 4x4 block grid
__device__ __forceinline__ void lower_block(int job, int& bi, int& bj) {
  bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= job) ++bi;
  bj = job - bi * (bi + 1) / 2;
}

// lambda_max of the symmetric M (full, ld SN) restricted to its leading n x n block
// by 60 power iterations from the all-ones vector; x, y: LDS vectors of SN.
__device__ double power_lmax(const double* M, int n, double* x, double* y, double* sh, int tid) {
  if (tid < SN) x[tid] = (tid < n) ? 1.0 / sqrt((double)n) : 0.0;
  __syncthreads();
  double nrm = 0.0;
  for (int it = 0; it < 60; ++it) {
    if (tid < SN) {
      double s = 0.0;
      for (int j = 0; j < SN; ++j) s += M[tid * SN + j] * x[j];
      y[tid] = s;
    }
    __syncthreads();
    const double v = (tid < n) ? y[tid] * y[tid] : 0.0;
    nrm = sqrt(block_sum(v, sh));
    if (tid < SN) x[tid] = (tid < n) ? y[tid] / nrm : 0.0;
    __syncthreads();
  }
  return nrm;
}

// the next problem of the queue, the same in every thread of the workgroup
__device__ __forceinline__ int next_problem(int* next, int* slot, int tid) {
  __syncthreads();
  if (tid == 0) *slot = atomicAdd(next, 1);
  __syncthreads();
  return *slot;
}

__global__ void set_counter_kernel(int* next, int value) { *next = value; }

__global__ __launch_bounds__(256) void pista_small_kernel(SmallParams p) {
  __shared__ double a[SN][SLD];  // factor / inverse
  __shared__ double b[SN][SLD];  // A Z A operand
  __shared__ double dl[SN];      // diag of the factor of the current A
  __shared__ double xv[SN], yv[SN];
  __shared__ double sh[4];
  __shared__ int taken;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* const S = p.ws + (int64_t)blockIdx.x * 6 * SNN;
  // the current iterate and the trial point; an accepted trial exchanges the two
  double* A = S + SNN;
  double* At = A + SNN;
  double* const W = S + 3 * SNN;
  double* const Z = W + SNN;
  double* const P = Z + SNN;
  int8_t* const GM = p.gm + (int64_t)blockIdx.x * SNN;

  for (int prob = blockIdx.x; prob < p.count; prob = next_problem(p.next, &taken, tid)) {
    const SmallProblem pr = p.prob[prob];
    SmallOut o = {};
    const int n = (int)pr.n;
    const double lam = pr.lam;

    // S (lower triangle read, stored full, zero padding); reject non-finite
    // entries and S_ii + lam <= 0
    double bad = 0.0;
    for (int e = tid; e < SNN; e += 256) {
      const int i = e / SN, j = e % SN;
      double v = 0.0;
      if (i < n && j < n) {
        v = pr.S[(int64_t)max(i, j) * n + min(i, j)];
        if (!(fabs(v) <= DBL_MAX)) bad += 1.0;
        if (i == j && !(v + lam > 0.0)) bad += 1.0;
      }
      S[e] = v;
    }
    if (block_sum(bad, sh) > 0.0) {
      o.error = 2;
      if (tid == 0) p.out[prob] = o;
      continue;
    }
    // A^(0): warm start or diag(1/(S_ii + lam)); identity in the padding
    for (int e = tid; e < SNN; e += 256) {
      const int i = e / SN, j = e % SN;
      double v;
      if (i < n && j < n)
        v = p.warm_start ? pr.A[(int64_t)max(i, j) * n + min(i, j)] : (i == j ? 1.0 / (S[e] + lam) : 0.0);
      else
        v = (i == j) ? 1.0 : 0.0;
      A[e] = v;
      if (j <= i) a[i][j] = v;
    }
    __syncthreads();
    if (lds_potrf<SN>(a, tid) >= 0) {
      o.error = p.warm_start ? 1 : 3;
      if (tid == 0) p.out[prob] = o;
      __syncthreads();
      continue;
    }
    if (tid < SN) dl[tid] = a[tid][tid];
    __syncthreads();

    o.status = GLASSO_MAX_ITER_DEV;
    for (;;) {
      // log det A from the factor in a
      const double ld = 2.0 * block_sum(tid < n ? log(dl[tid]) : 0.0, sh);
      // a1: W = inv(L)^T inv(L), written full
      lds_trtri<SN>(a, tid);
      for (int job = wave; job < 10; job += 4) {
        int bi, bj;
        lower_block(job, bi, bj);
        const v4d acc = lauum_block(a, bi, bj, lane);
        for_block(acc, lane, [&](int r, int c, double v) {
          const int i = 16 * bi + r, j = 16 * bj + c;
          if (bi != bj || c <= r) {
            W[i * SN + j] = v;
            W[j * SN + i] = v;
          }
        });
      }
      __syncthreads();
      // a2: gradient pass over the lower triangle (weights 1 on, 2 off the diagonal);
      // all of a thread's elements are read and computed before any is stored, so
      // the loads are not serialised behind stores the compiler cannot disambiguate
      double s_absz = 0.0, s_z2 = 0.0, m_absz = 0.0, s_absa = 0.0, s_nnz = 0.0, s_sa = 0.0;
      constexpr int CH = 4;  // elements per chunk: e = tid + 256 k
#pragma unroll 1
      for (int k0 = 0; k0 < SNN / 256; k0 += CH) {
        double zv[CH];
        int8_t gv[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int e = tid + 256 * (k0 + k), i = e / SN, j = e % SN;
          zv[k] = 0.0;
          gv[k] = 0;
          if (j <= i && i < n) {
            const double av = A[e], s = S[e];
            grad_element(av, s, W[e], lam, zv[k], gv[k]);
            const double z = zv[k];
            const double wgt = (i == j) ? 1.0 : 2.0;
            s_absz += wgt * fabs(z);
            s_z2 += wgt * (z * z);
            m_absz = fmax(m_absz, fabs(z));
            s_absa += wgt * fabs(av);
            s_nnz += (av != 0.0) ? wgt : 0.0;
            s_sa += wgt * (s * av);
          }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int e = tid + 256 * (k0 + k), i = e / SN, j = e % SN;
          if (j > i) continue;
          Z[e] = zv[k];
          Z[j * SN + i] = zv[k];
          GM[e] = gv[k];
          GM[j * SN + i] = gv[k];
        }
      }
      const double sz = block_sum(s_absz, sh);
      const double sz2 = block_sum(s_z2, sh);
      const double mz = block_max(m_absz, sh);
      const double sa = block_sum(s_absa, sh);
      const double nnz = block_sum(s_nnz, sh);
      const double ssa = block_sum(s_sa, sh);
      o.objective = -ld + ssa + lam * sa;
      o.kkt_rel1 = sz / sa;
      o.kkt_fro = sqrt(sz2);
      o.kkt_max = mz;
      o.nnz = nnz;
      if (o.kkt_rel1 <= p.tol) {
        o.status = GLASSO_CONVERGED_DEV;
        break;
      }
      if (o.iterations >= p.max_iter) break;
      // a3: X = A Z (A in a, Z in b), then P = tril(X A) (X in b)
      for (int e = tid; e < SNN; e += 256) {
        const int i = e / SN, j = e % SN;
        a[i][j] = A[e];
        b[i][j] = Z[e];
      }
      __syncthreads();
      v4d xacc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) xacc[q] = nn_block(a, b, wave, q, lane);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q)
        for_block(xacc[q], lane, [&](int r, int c, double v) { b[16 * wave + r][16 * q + c] = v; });
      __syncthreads();
      for (int job = wave; job < 10; job += 4) {
        int bi, bj;
        lower_block(job, bi, bj);
        const v4d acc = nn_block(b, a, bi, bj, lane);
        for_block(acc, lane, [&](int r, int c, double v) { P[(16 * bi + r) * SN + 16 * bj + c] = v; });
      }
      __syncthreads();
      // a4-a6: trials t = t0, t0*shrink, ... until PD with a strict decrease
      double t = p.t0;
      bool fb_used = false, accepted = false;
      for (;;) {
        if (t < p.t_floor && !fb_used) {
          const double pa = power_lmax(A, n, xv, yv, sh, tid);
          const double pw = power_lmax(W, n, xv, yv, sh, tid);
          const double cond = (1.05 * pa) * (1.05 * pw);
          const double tf = (0.9 / cond) * (0.9 / cond);
          t = (tf < t) ? tf : t;
          fb_used = true;
          ++o.fallback_steps;
        }
        if (t < p.t_min) break;
        double s_tr = 0.0, s_l1 = 0.0, s_w = 0.0;
        constexpr int CHT = 4;
#pragma unroll 1
        for (int k0 = 0; k0 < SNN / 256; k0 += CHT) {
          double atv[CHT];
#pragma unroll
          for (int k = 0; k < CHT; ++k) {
            const int e = tid + 256 * (k0 + k), i = e / SN, j = e % SN;
            double at = 0.0;
            if (j <= i) {
              if (i < n) {
                const int8_t gm = GM[e];
                if (gm != 0) {
                  const double av = A[e];
                  const double Cij = c_element(i == j, A[i * SN + i], A[j * SN + j], av, lam);
                  at = trial_element(av, P[e], Cij, (double)gm, t);
                  const double wgt = (i == j) ? 1.0 : 2.0;
                  s_tr += wgt * (S[e] * (at - av));
                  s_l1 += wgt * (fabs(at) - fabs(av));
                  if (p.sigma > 0.0) s_w += wgt * (W[e] * (at - av));
                }
              } else {
                at = (i == j) ? 1.0 : 0.0;
              }
            }
            atv[k] = at;
          }
#pragma unroll
          for (int k = 0; k < CHT; ++k) {
            const int e = tid + 256 * (k0 + k), i = e / SN, j = e % SN;
            if (j > i) continue;
            At[e] = atv[k];
            At[j * SN + i] = atv[k];
            a[i][j] = atv[k];
          }
        }
        const double dtr = block_sum(s_tr, sh);
        const double dl1 = block_sum(s_l1, sh);
        // sufficient decrease: sigma times <g, At - A> + lam (||At||_1 - ||A||_1), g = S - W
        const double target = (p.sigma > 0.0) ? p.sigma * ((dtr - block_sum(s_w, sh)) + lam * dl1) : 0.0;
        ++o.ls_trials;
        const int fail = lds_potrf<SN>(a, tid);
        bool ok = false;
        if (fail < 0) {
          const double dlog = 2.0 * block_sum(tid < n ? log(dl[tid] / a[tid][tid]) : 0.0, sh);
          ok = (dlog + dtr + lam * dl1) < target;
        }
        __syncthreads();
        if (ok) {
          // a7: A <- At by exchanging the two buffers; the factor of At stays in a
          double* const tmp = A;
          A = At;
          At = tmp;
          if (tid < SN) dl[tid] = a[tid][tid];
          __syncthreads();
          ++o.iterations;
          accepted = true;
          break;
        }
        t *= p.shrink;
      }
      if (!accepted) {
        o.status = GLASSO_LS_FAILED_DEV;
        break;
      }
    }
    // outputs: A (full) and W of the final iterate
    for (int e = tid; e < n * n; e += 256) {
      const int i = e / n, j = e % n;
      pr.A[e] = A[i * SN + j];
      if (pr.W) pr.W[e] = W[i * SN + j];
    }
    if (tid == 0) p.out[prob] = o;
    __syncthreads();
  }
}

}  // namespace

int solve_small(hipStream_t stream, const SmallParams& p, int grid) {
  if (p.count <= 0) return 0;
  if (grid <= 0) return -1;
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(1), 0, stream, p.next, grid);
  hipLaunchKernelGGL(pista_small_kernel, dim3(grid), dim3(256), 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
