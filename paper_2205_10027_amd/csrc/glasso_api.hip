// C ABI of libglasso: handle, workspace and the pISTA driver (Alg. 1 with the
// Sec. 5 initialisation, line search and stopping rule).  Every arithmetic step
// runs in the kernels of gemm_f64.hip, chol.hip and passes.hip; the host only
// sequences launches and reads back a few scalars (KKT, decrease, pivot status).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>

#include "../../include/glasso.h"
#include "common.h"
#include "kernels.h"

using namespace glasso;

namespace {

constexpr int FLAG_FACTOR = 0;  // info of the latest Cholesky
constexpr int NFLAGS = 16;

struct Workspace {
  int64_t cap = 0;  // padded size the buffers were laid out for
  int64_t np = 0;   // padded size (leading dimension) of the current problem
  void* base = nullptr;
  size_t bytes = 0;
  double *S = nullptr, *A = nullptr, *At = nullptr, *L = nullptr, *Lt = nullptr, *W = nullptr, *Z = nullptr,
         *X = nullptr, *P = nullptr;
  int8_t* GM = nullptr;
  double *dL = nullptr, *dLt = nullptr, *Dinv = nullptr, *Dinvt = nullptr;
  double* part = nullptr;
  double* scal = nullptr;
  int* flags = nullptr;
  int64_t* bad = nullptr;
  double* vec = nullptr;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Carve the workspace of padded size np out of one allocation (base may be null
// to only measure).
size_t layout(Workspace& w, int64_t np, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const size_t mat = (size_t)np * np * sizeof(double);
  w.S = (double*)take(mat);
  w.A = (double*)take(mat);
  w.At = (double*)take(mat);
  w.L = (double*)take(mat);
  w.Lt = (double*)take(mat);
  w.W = (double*)take(mat);
  w.Z = (double*)take(mat);
  w.X = (double*)take(mat);
  w.P = (double*)take(mat);
  w.GM = (int8_t*)take((size_t)np * np);
  w.dL = (double*)take(np * sizeof(double));
  w.dLt = (double*)take(np * sizeof(double));
  w.Dinv = (double*)take((size_t)np * TILE * sizeof(double));
  w.Dinvt = (double*)take((size_t)np * TILE * sizeof(double));
  w.part = (double*)take((size_t)pass_tiles(np) * 8 * sizeof(double));
  w.scal = (double*)take(SC_COUNT * sizeof(double));
  w.flags = (int*)take(NFLAGS * sizeof(int));
  w.bad = (int64_t*)take(sizeof(int64_t));
  w.vec = (double*)take(2 * np * sizeof(double));
  return off;
}

}  // namespace

struct glasso_handle_s {
  glasso_options opt;
  int device = 0;
  Workspace ws;
  double* host = nullptr;  // pinned: scalars + flags
  hipEvent_t ev[6] = {};
};

namespace {

#define HIP_TRY(expr)                                  \
  do {                                                 \
    if ((expr) != hipSuccess) return GLASSO_ERR_HIP;   \
  } while (0)
#define K_TRY(expr)                                    \
  do {                                                 \
    int _rc = (expr);                                  \
    if (_rc == -1) return GLASSO_ERR_INTERNAL;         \
    if (_rc) return GLASSO_ERR_HIP;                    \
  } while (0)

glasso_err ensure_workspace(glasso_handle h, int64_t np) {
  Workspace& w = h->ws;
  if (w.base && w.cap >= np) {
    w.np = np;
    return GLASSO_OK;
  }
  if (w.base) {
    (void)hipFree(w.base);
    w = Workspace();
  }
  Workspace probe;
  const size_t bytes = layout(probe, np, nullptr);
  void* base = nullptr;
  if (hipMalloc(&base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return GLASSO_ERR_OOM;
  }
  if (hipMemset(base, 0, bytes) != hipSuccess) {
    (void)hipFree(base);
    return GLASSO_ERR_HIP;
  }
  layout(w, np, (char*)base);
  w.base = base;
  w.bytes = bytes;
  w.cap = np;
  w.np = np;
  return GLASSO_OK;
}

// copy the device scalar slots and flags to pinned host memory and wait
glasso_err fetch(glasso_handle h, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(h->host, h->ws.scal, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(h->host + SC_COUNT, h->ws.flags, NFLAGS * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}
int host_flag(glasso_handle h, int i) { return reinterpret_cast<int*>(h->host + SC_COUNT)[i]; }

glasso_err check_options(const glasso_options* o) {
  if (o->precision != GLASSO_FP64 && o->precision != GLASSO_MIXED_FP32) return GLASSO_ERR_INVALID_ARG;
  if (o->max_iter < 0) return GLASSO_ERR_INVALID_ARG;
  if (!(o->t0 > 0.0) || !(o->shrink > 0.0 && o->shrink < 1.0) || !(o->t_floor >= 0.0) || !(o->t_min > 0.0))
    return GLASSO_ERR_INVALID_ARG;
  return GLASSO_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

// Factor the padded matrix in w.L (lower, in place) and wait for the pivot status.
glasso_err factor_current(glasso_handle h, hipStream_t st, int* info_out) {
  Workspace& w = h->ws;
  HIP_TRY(hipMemsetAsync(w.flags + FLAG_FACTOR, 0, sizeof(int), st));
  K_TRY(potrf_lower(st, w.L, w.np, (int)w.np, w.dL, w.Dinv, w.flags + FLAG_FACTOR));
  glasso_err e = fetch(h, st);
  if (e) return e;
  *info_out = host_flag(h, FLAG_FACTOR);
  return GLASSO_OK;
}

// W (lower) = A^{-1} from the factor in w.L: L <- inv(L) in place, W = inv(L)^T inv(L).
glasso_err inverse_from_factor(Workspace& w, hipStream_t st) {
  K_TRY(trtri_lower(st, w.L, w.np, (int)w.np, w.Dinv, w.X, nullptr));
  K_TRY(lauum_lower(st, w.L, w.np, w.W, w.np, (int)w.np));
  return GLASSO_OK;
}

// P (lower) = A Z A: X = A Z^T (Z symmetric), P = tril(X A^T) (A symmetric).
// Mixed FP32: A and Z are rounded to FP32 (A32, Z32 in the X buffer), X32 = A32 Z32^T
// overwrites Z (no longer needed), P = tril(X32 A32^T) is written in FP64.
glasso_err precond_product(Workspace& w, hipStream_t st, int precision) {
  const int np = (int)w.np;
  if (precision == GLASSO_FP64) {
    K_TRY(gemm_f64(st, 0, 0, np, np, np, 1.0, w.A, np, w.Z, np, 0.0, w.X, np, 0, 0, 0, nullptr, 1, 0, 0, 0, 1));
    K_TRY(gemm_f64(st, 0, 0, np, np, np, 1.0, w.X, np, w.A, np, 0.0, w.P, np, 1, 0, 0, nullptr, 1, 0, 0, 0, 1));
    return GLASSO_OK;
  }
  if (precision == GLASSO_MIXED_FP32) {
    const int64_t nn = (int64_t)np * np;
    float* A32 = reinterpret_cast<float*>(w.X);
    float* Z32 = A32 + nn;
    float* X32 = reinterpret_cast<float*>(w.Z);
    K_TRY(f64_to_f32(st, w.A, A32, nn));
    K_TRY(f64_to_f32(st, w.Z, Z32, nn));
    K_TRY(gemm_f32_nt(st, np, np, np, A32, np, Z32, np, X32, np, 0, 0));
    K_TRY(gemm_f32_nt(st, np, np, np, X32, np, A32, np, w.P, np, 1, 1));
    return GLASSO_OK;
  }
  return GLASSO_ERR_INVALID_ARG;
}

// cond(A) ~ lambda_max(A) * lambda_max(A^{-1}) by power iteration; t = (0.9/cond)^2.
// Ritz values approach from below, so each estimate is inflated by 5%.
glasso_err cond_fallback_step(glasso_handle h, hipStream_t st, int64_t n, double* t_out) {
  Workspace& w = h->ws;
  K_TRY(power_iteration(st, w.A, n, w.np, w.vec, w.scal + SC_POWER_A, 60));
  HIP_TRY(hipMemcpyAsync(w.X, w.W, (size_t)w.np * w.np * sizeof(double), hipMemcpyDeviceToDevice, st));
  K_TRY(mirror_lower(st, w.X, w.np));
  K_TRY(power_iteration(st, w.X, n, w.np, w.vec, w.scal + SC_POWER_W, 60));
  glasso_err e = fetch(h, st);
  if (e) return e;
  const double cond = (1.05 * h->host[SC_POWER_A]) * (1.05 * h->host[SC_POWER_W]);
  *t_out = (0.9 / cond) * (0.9 / cond);
  return GLASSO_OK;
}

}  // namespace

extern "C" {

glasso_err glasso_default_options(glasso_options* opt) {
  if (!opt) return GLASSO_ERR_INVALID_ARG;
  memset(opt, 0, sizeof(*opt));
  opt->precision = GLASSO_FP64;
  opt->max_iter = 500;
  opt->t0 = 1.0;
  opt->shrink = 0.5;
  opt->t_floor = 1e-4;
  opt->t_min = 1e-12;
  opt->warm_start = 0;
  return GLASSO_OK;
}

glasso_err glasso_create(glasso_handle* h, const glasso_options* opt) {
  if (!h) return GLASSO_ERR_INVALID_ARG;
  *h = nullptr;
  glasso_options o;
  if (opt)
    o = *opt;
  else
    glasso_default_options(&o);
  if (check_options(&o)) return GLASSO_ERR_INVALID_ARG;
  glasso_handle_s* hh = new (std::nothrow) glasso_handle_s();
  if (!hh) return GLASSO_ERR_OOM;
  hh->opt = o;
  if (hipGetDevice(&hh->device) != hipSuccess) {
    delete hh;
    return GLASSO_ERR_HIP;
  }
  if (hipHostMalloc((void**)&hh->host, (SC_COUNT + NFLAGS) * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete hh;
    return GLASSO_ERR_HIP;
  }
  for (auto& e : hh->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipHostFree(hh->host);
      delete hh;
      return GLASSO_ERR_HIP;
    }
  }
  *h = hh;
  return GLASSO_OK;
}

glasso_err glasso_destroy(glasso_handle h) {
  if (!h) return GLASSO_OK;
  if (h->ws.base) (void)hipFree(h->ws.base);
  if (h->host) (void)hipHostFree(h->host);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
  return GLASSO_OK;
}

const char* glasso_error_string(glasso_err e) {
  switch (e) {
    case GLASSO_OK: return "success";
    case GLASSO_ERR_INVALID_ARG: return "invalid argument";
    case GLASSO_ERR_NOT_PD: return "matrix is not positive definite";
    case GLASSO_ERR_OOM: return "out of device memory";
    case GLASSO_ERR_HIP: return "HIP runtime error";
    case GLASSO_ERR_INTERNAL: return "internal error";
  }
  return "unknown error";
}

glasso_err glasso_workspace_size(int64_t n, int precision, size_t* bytes) {
  if (n < 1 || !bytes || precision < GLASSO_FP64 || precision > GLASSO_MIXED_BF16X3) return GLASSO_ERR_INVALID_ARG;
  Workspace probe;
  *bytes = layout(probe, pad_to_tile(n), nullptr);
  return GLASSO_OK;
}

glasso_err glasso_solve(glasso_handle h, const double* S, int64_t n, double lambda, double tol, double* A,
                        double* W, glasso_info* info, void* stream) {
  if (!h || !S || !A || n < 1 || !(lambda > 0.0) || !(tol > 0.0) || !isfinite(lambda) || n > (1 << 20))
    return GLASSO_ERR_INVALID_ARG;
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t st = (hipStream_t)stream;
  const glasso_options& o = h->opt;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, np);
  if (e) return e;
  Workspace& w = h->ws;

  // S into the padded layout; reject non-finite entries and S_ii + lambda <= 0
  HIP_TRY(hipMemsetAsync(w.bad, 0, sizeof(int64_t), st));
  K_TRY(copy_in_padded(st, S, n, w.S, np, w.bad, lambda, 1));
  int64_t nbad = 0;
  HIP_TRY(hipMemcpyAsync(&nbad, w.bad, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (nbad) return GLASSO_ERR_INVALID_ARG;

  // A^(0): warm start or diag(1/(S_ii + lambda)) (Sec. 5); its factor
  if (o.warm_start)
    K_TRY(pad_copy_f64(st, A, n, np, w.A, w.L, 1));
  else
    K_TRY(init_diag(st, w.S, n, np, lambda, w.A, w.L));
  int finfo = 0;
  e = factor_current(h, st, &finfo);
  if (e) return e;
  if (finfo) return o.warm_start ? GLASSO_ERR_NOT_PD : GLASSO_ERR_INVALID_ARG;

  const int tiles = (int)pass_tiles(np);
  int it = 0, trials = 0, fallbacks = 0;
  int status = GLASSO_MAX_ITER;
  double phase[8] = {0};
  for (;;) {
    // a1: W = A^{-1} from the accepted factor
    HIP_TRY(hipEventRecord(h->ev[0], st));
    e = inverse_from_factor(w, st);
    if (e) return e;
    HIP_TRY(hipEventRecord(h->ev[1], st));
    // a2: gradient, free set, sign guess, Z and the KKT measure
    K_TRY(pass_grad(st, w.S, w.W, w.A, w.dL, n, n, np, lambda, w.Z, w.GM, w.part, w.scal));
    HIP_TRY(hipEventRecord(h->ev[2], st));
    e = fetch(h, st);
    if (e) return e;
    phase[1] += elapsed(h->ev[0], h->ev[1]);
    phase[2] += elapsed(h->ev[1], h->ev[2]);
    const double kkt = h->host[SC_KKT_REL1];
    if (kkt <= tol) {
      status = GLASSO_CONVERGED;
      break;
    }
    if (it >= o.max_iter) {
      status = GLASSO_MAX_ITER;
      break;
    }
    // a3: P = A Z A
    HIP_TRY(hipEventRecord(h->ev[2], st));
    e = precond_product(w, st, o.precision);
    if (e) return e;
    HIP_TRY(hipEventRecord(h->ev[3], st));
    // a4-a6: trial points t = t0, t0*shrink, ... until PD with a strict decrease
    double t = o.t0;
    bool fallback = false, accepted = false;
    for (;;) {
      if (t < o.t_floor && !fallback) {
        double tf = 0.0;
        e = cond_fallback_step(h, st, n, &tf);
        if (e) return e;
        t = std::min(t, tf);
        fallback = true;
        ++fallbacks;
      }
      if (t < o.t_min) break;
      K_TRY(pass_trial(st, w.A, w.P, w.S, w.GM, n, np, lambda, t, w.At, w.Lt, w.part, w.flags + FLAG_FACTOR));
      K_TRY(potrf_lower(st, w.Lt, np, (int)np, w.dLt, w.Dinvt, w.flags + FLAG_FACTOR));
      K_TRY(finish_trial(st, w.part, tiles, w.dL, w.dLt, w.flags + FLAG_FACTOR, n, lambda, w.scal));
      e = fetch(h, st);
      if (e) return e;
      ++trials;
      if (host_flag(h, FLAG_FACTOR) == 0 && h->host[SC_DF] < 0.0) {
        accepted = true;
        break;
      }
      t *= o.shrink;
    }
    HIP_TRY(hipEventRecord(h->ev[4], st));
    HIP_TRY(hipEventSynchronize(h->ev[4]));
    phase[3] += elapsed(h->ev[2], h->ev[3]);
    phase[4] += elapsed(h->ev[3], h->ev[4]);
    if (!accepted) {
      status = GLASSO_LS_FAILED;
      break;
    }
    // a7: accept
    std::swap(w.A, w.At);
    std::swap(w.L, w.Lt);
    std::swap(w.dL, w.dLt);
    std::swap(w.Dinv, w.Dinvt);
    ++it;
  }

  K_TRY(sym_copy_out(st, w.A, np, A, n, 0));
  if (W) K_TRY(sym_copy_out(st, w.W, np, W, n, 1));
  HIP_TRY(hipStreamSynchronize(st));
  if (info) {
    memset(info, 0, sizeof(*info));
    info->objective = h->host[SC_OBJECTIVE];
    info->kkt_rel1 = h->host[SC_KKT_REL1];
    info->kkt_fro = h->host[SC_KKT_FRO];
    info->kkt_max = h->host[SC_MAX_ABS_Z];
    info->nnz = (int64_t)llround(h->host[SC_NNZ_A]);
    info->iterations = it;
    info->ls_trials = trials;
    info->status = status;
    info->fallback_steps = fallbacks;
    for (int i = 1; i < 8; ++i) info->time_ms[i] = phase[i];
    info->time_ms[0] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  return GLASSO_OK;
}

// ------------------------------------------------------------------ step-level entry points
glasso_err glasso_cholesky(glasso_handle h, const double* A, int64_t n, double* L, int64_t* info, double* logdet,
                           void* stream) {
  if (!h || !A || !L || n < 1) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, np);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.L, nullptr, 1));
  int finfo = 0;
  e = factor_current(h, st, &finfo);
  if (e) return e;
  if (info) *info = finfo;
  K_TRY(sym_copy_out(st, w.L, np, L, n, 2));
  if (logdet) {
    K_TRY(sum_log(st, w.dL, n, w.scal + SC_LOGDET));
    e = fetch(h, st);
    if (e) return e;
    *logdet = finfo ? NAN : h->host[SC_LOGDET];
  }
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

glasso_err glasso_inverse(glasso_handle h, const double* A, int64_t n, double* W, void* stream) {
  if (!h || !A || !W || n < 1) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, np);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.L, nullptr, 1));
  int finfo = 0;
  e = factor_current(h, st, &finfo);
  if (e) return e;
  if (finfo) return GLASSO_ERR_NOT_PD;
  e = inverse_from_factor(w, st);
  if (e) return e;
  K_TRY(sym_copy_out(st, w.W, np, W, n, 1));
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

glasso_err glasso_gradient_pass(glasso_handle h, const double* S, const double* W, const double* A, int64_t n,
                                double lambda, double* Z, int8_t* GM, double* kkt, void* stream) {
  if (!h || !S || !W || !A || !Z || !GM || n < 1 || !(lambda > 0.0)) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, np);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, S, n, np, w.S, nullptr, 0));
  K_TRY(pad_copy_f64(st, W, n, np, w.W, nullptr, 1));
  K_TRY(pad_copy_f64(st, A, n, np, w.A, nullptr, 1));
  // no factor is at hand here: the log-det term is left out (nlog = 0)
  K_TRY(pass_grad(st, w.S, w.W, w.A, w.dL, n, 0, np, lambda, w.Z, w.GM, w.part, w.scal));
  K_TRY(sym_copy_out(st, w.Z, np, Z, n, 0));
  K_TRY(unpad_copy_i8(st, w.GM, np, GM, n));
  e = fetch(h, st);
  if (e) return e;
  if (kkt) {
    kkt[0] = h->host[SC_SUM_ABS_Z];
    kkt[1] = h->host[SC_SUM_ABS_A];
    kkt[2] = h->host[SC_KKT_FRO];
    kkt[3] = h->host[SC_MAX_ABS_Z];
  }
  return GLASSO_OK;
}

glasso_err glasso_precond_product(glasso_handle h, const double* A, const double* Z, int64_t n, int precision,
                                  double* P, void* stream) {
  if (!h || !A || !Z || !P || n < 1) return GLASSO_ERR_INVALID_ARG;
  if (precision != GLASSO_FP64 && precision != GLASSO_MIXED_FP32) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, np);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.A, nullptr, 1));
  K_TRY(pad_copy_f64(st, Z, n, np, w.Z, nullptr, 0));
  e = precond_product(w, st, precision);
  if (e) return e;
  K_TRY(sym_copy_out(st, w.P, np, P, n, 1));
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

glasso_err glasso_trial_point(glasso_handle h, const double* A, const double* P, const double* S, const int8_t* GM,
                              int64_t n, double lambda, double t, double* At, double* sums, void* stream) {
  if (!h || !A || !P || !S || !GM || !At || n < 1 || !(lambda > 0.0) || !(t > 0.0)) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, np);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.A, nullptr, 1));
  K_TRY(pad_copy_f64(st, P, n, np, w.P, nullptr, 0));
  K_TRY(pad_copy_f64(st, S, n, np, w.S, nullptr, 0));
  K_TRY(pad_copy_i8(st, GM, n, np, w.GM));
  K_TRY(pass_trial(st, w.A, w.P, w.S, w.GM, n, np, lambda, t, w.At, w.Lt, w.part, w.flags + FLAG_FACTOR));
  // no factor: the log-ratio term reads the same diagonal twice and vanishes
  K_TRY(finish_trial(st, w.part, (int)pass_tiles(np), w.dL, w.dL, w.flags + FLAG_FACTOR, 0, lambda, w.scal));
  K_TRY(sym_copy_out(st, w.At, np, At, n, 0));
  e = fetch(h, st);
  if (e) return e;
  if (sums) {
    sums[0] = h->host[SC_DTR];
    sums[1] = h->host[SC_DL1];
  }
  return GLASSO_OK;
}

}  // extern "C"
