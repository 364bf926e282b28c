// Per-element formulas of the gradient and trial passes and the fixed-order
// workgroup reductions, shared by the blocked passes and the persistent
// small-problem solver.  Included with floating-point contraction disabled, so
// every element is computed with the same IEEE operations as the plain formulas.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace glasso {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Sum (or max) over a 256-thread block in a fixed order; result valid in every thread.
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}
__device__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__device__ __forceinline__ double sign_of(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// Gradient-pass element (Sec. 4.1): g = S - W, M = (A != 0) | (|g| > lam),
// G = sign(A) or -sign(g); z = (g + lam G) on M (the minimum-norm subgradient),
// gm = G on M; both 0 off the free set.
__device__ __forceinline__ void grad_element(double a, double s, double w, double lam, double& z, int8_t& gm) {
  const double g = s - w;
  const bool nz = (a != 0.0);
  const double G = nz ? sign_of(a) : -sign_of(g);
  const bool M = nz || (fabs(g) > lam);
  z = 0.0;
  gm = 0;
  if (M) {
    z = g + lam * G;
    gm = (int8_t)G;
  }
}

// eq. c: C_ij = lam (A_ii A_jj + A_ij^2) off the diagonal, lam A_ii^2 on it
__device__ __forceinline__ double c_element(bool on_diag, double aii, double ajj, double a, double lam) {
  return on_diag ? lam * (aii * aii) : lam * ((aii * ajj) + (a * a));
}

// Trial element on the free set (eqs. b, d_sol): B = P - C G, At = ST(A - tB, tC)
__device__ __forceinline__ double trial_element(double a, double p, double Cij, double gm, double t) {
  const double B = p - Cij * gm;
  const double x = a - t * B;
  const double tau = t * Cij;
  const double m = fmax(fabs(x) - tau, 0.0);
  return sign_of(x) * m;
}

// G-ISTA trial element (eq. proximal_gen with H = I, the proximal-gradient step):
// At = ST(A - t g, t lam) with g = S - W.  Off the free set (A = 0, |g| <= lam) it is
// exactly 0, so the pass visits only the free set, as for the pISTA step.
__device__ __forceinline__ double gista_element(double a, double s, double w, double lam, double t) {
  const double g = s - w;
  const double x = a - t * g;
  const double tau = t * lam;
  const double m = fmax(fabs(x) - tau, 0.0);
  return sign_of(x) * m;
}

}  // namespace

}  // namespace glasso
